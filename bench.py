"""Benchmark: milliseconds per fast flow-based cartogram iteration on one GPU.

One step = one FFB iteration of the whole hot path on the L = 1024 workload
(600-region seeded Voronoi map, Pareto(1.2) densities clipped at 1e3, 1.0 M
polygon vertices plus all 1024^2 grid nodes advected): areas, density grid,
blur + flux transforms, adaptive Dormand-Prince advection of every point to
t = 1, areas and relative errors.  Each step starts from the same resident
input map (a device-to-device copy of the points, inside the timed region),
so every step does the same work.  Inputs are resident in HBM before timing.

Second part of the metric (fwd+bwd / fwd): on the L = 512, 50-region map,
three rounds (blur widths 4, 2, 1) of the full cartogram (100 k vertices and
all 512^2 grid nodes) without recording, against the same three rounds
recorded plus the reverse pass that yields the gradient of the area loss
with respect to the 50 region statistics.

Printed: one JSON line with the metric, the roofline of the dominant kernel
(the advection launch, timed with events on its stream around the whole
integration call, so the ~45 us point sort by cell that precedes the launch
counts against it) and the FP64 oracle
timed on the host cores on a bounded sample.
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

HBM_PEAK_GBS = 8000.0

# HBM bytes per RK attempt of the advection launch on the L = 1024 workload,
# from FETCH_SIZE and WRITE_SIZE counter runs calibrated on a copy of known
# size, for the kernel source with this sha256 prefix; reported only while the
# source is unchanged.
ADVECT_TRAFFIC = {"bytes_per_attempt": 2.2811e+10 / 267,
                  "valu_wave_insts_per_attempt": 2.9315e+09 / 267,
                  "workload": "c3_L1024", "source_sha256": "258649db088c6f02"}
# non-packed FP32 issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3_L1024")
    ap.add_argument("--sigma", type=float, default=4.0)
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="time whole oracle iterations until this much work is timed")
    ap.add_argument("--no-cpu-single", dest="cpu_single", action="store_false",
                    help="skip the single-core timing of the oracle")
    ap.add_argument("--no-loop", action="store_true",
                    help="skip the loop to < 1%% error")
    ap.add_argument("--no-grad", action="store_true",
                    help="skip the fwd+bwd / fwd measurement")
    ap.add_argument("--grad-steps", type=int, default=10)
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-maps measurement")
    ap.add_argument("--batch-maps", type=int, default=256)
    ap.add_argument("--no-rect", action="store_true",
                    help="skip the rectangular map with holes and multipolygons")
    ap.add_argument("--no-diffusion", action="store_true",
                    help="skip the diffusion-cartogram comparison")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import synth
    import paper_1802_07625_amd as ffb

    if not os.path.exists(ffb.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    m = synth.workload(args.workload)
    L = m.lx
    pts_h = np.concatenate([m.xy, synth.grid_nodes(L, L)]).astype(np.float32)
    P, V = pts_h.shape[0], m.n_vertices
    print(f"# workload {args.workload}: L={L} regions={m.n_regions} V={V} P={P} E={m.n_entries}",
          file=sys.stderr, flush=True)
    pts0 = torch.as_tensor(pts_h, device=dev)
    pts = pts0.clone()
    geom = ffb.Geometry.from_map(m, xy=pts[:V])
    value = torch.as_tensor(m.value, dtype=torch.float64, device=dev)
    ctx = ffb.Context(L, L, max_points=P)
    opts = ffb.IntegrateOpts(tol=args.tol)
    stream = torch.cuda.current_stream()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    # whole-step events, for the median step time
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    stats_all = torch.zeros((max(args.steps, 1), 4), dtype=torch.int32, device=dev)

    def step(i=None):
        if i is not None:
            evs[i][0].record(stream)
        pts.copy_(pts0)
        area0, _, _ = ctx.area_error(geom, value)
        rho, pad = ctx.density(geom, value, area0)
        fields, rb = ctx.flux(rho, args.sigma)
        st = stats_all[i] if i is not None else None
        if i is not None:
            ev[i][0].record(stream)
        stats, _ = ctx.integrate(fields, rb, pts, opts, h_cap=0, stats=st)
        if i is not None:
            ev[i][1].record(stream)
        area1, err1, mx = ctx.area_error(geom, value)
        if i is not None:
            evs[i][1].record(stream)
        return stats, mx

    for _ in range(args.warmup):
        step()
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        stats, mx = step(i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.sync()
    ms_step = 1e3 * wall / args.steps
    adv_ms = np.array([a.elapsed_time(b) for a, b in ev])
    st = stats_all.cpu().numpy()
    attempts = st[:, 2].astype(np.float64)
    # algorithmic bytes of one advection launch: per RK attempt the point
    # state is read and written once (16 B per point) and the packed fields
    # are read once (16 B per node); S attempts per launch
    bytes_per_attempt = 16.0 * P + 16.0 * L * L
    achieved = float(np.mean(bytes_per_attempt * attempts / (adv_ms * 1e-3)) / 1e9)
    traffic, valu = None, None
    if args.workload == ADVECT_TRAFFIC["workload"] and _advect_sha() == ADVECT_TRAFFIC["source_sha256"]:
        traffic = round(float(np.mean(ADVECT_TRAFFIC["bytes_per_attempt"] * attempts
                                      / (adv_ms * 1e-3)) / 1e9), 1)
        lane_ops = float(np.mean(64 * ADVECT_TRAFFIC["valu_wave_insts_per_attempt"] * attempts
                                 / (adv_ms * 1e-3)))
        valu = {"achieved": round(lane_ops / 1e12, 2), "peak": round(VALU_PEAK_LANE_OPS / 1e12, 2),
                "unit": "T lane-instructions/s (non-packed FP32 issue)",
                "frac": round(lane_ops / VALU_PEAK_LANE_OPS, 4)}
    # the VALU view (SQ_INSTS_VALU per attempt from the counter run, times 64
    # lanes, over the measured attempt time) shows the bound that binds: the
    # kernel is instruction-issue bound, the byte model above is not
    result = {
        "metric": "ms per FFB iteration at L=1024 (FP32 vs FP64 oracle); fwd+bwd/fwd time",
        "value": round(ms_step, 4),
        "unit": "ms/iteration",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "L": L, "regions": m.n_regions,
                   "vertices": V, "points": P, "ring_entries": m.n_entries,
                   "densities": "pareto(1.2) clipped 1e3" if args.workload == "c3_L1024" else "",
                   "sigma": args.sigma, "tol": args.tol,
                   "point_order": "sorted by start cell inside ffb_integrate (timed)",
                   "rk_attempts_mean": float(attempts.mean()),
                   "rk_accepted_mean": float(st[:, 0].mean()),
                   "rk_rejected_mean": float(st[:, 1].mean()),
                   "ms_median_step": round(float(np.median(
                       [a.elapsed_time(b) for a, b in evs])), 4),
                   "advect_ms_mean": round(float(adv_ms.mean()), 4),
                   "us_per_attempt": round(float((adv_ms / attempts).mean() * 1e3), 3),
                   "final_max_area_error": float(mx)},
        "roofline": {"kernel": "k_advect", "bound": "hbm", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "bytes_per_attempt": bytes_per_attempt, "valu": valu},
    }

    if not args.no_loop:
        # the converging run: rounds with blur 4 * 2^-k until max |e_r| < 1 %;
        # the points are sorted by cell in round 0 and later rounds keep that
        # order (setting the option drops any order kept from before)
        ctx.set_option(ffb.OPT_POINT_ORDER, ffb.POINT_ORDER_KEEP)
        pts.copy_(pts0)
        torch.cuda.synchronize()
        rounds, mxv, t_loop = 0, None, time.perf_counter()
        area, round_ms, round_err, round_att = None, [], [], []
        for k in range(30):
            t_r = time.perf_counter()
            res = ffb.iterate(ctx, geom, value, pts, ffb.default_sigma(k), opts, area_before=area)
            area = res.area_after
            rounds += 1
            mxv = float(res.max_err_after)     # sync point once per round
            round_ms.append(round(1e3 * (time.perf_counter() - t_r), 3))
            round_err.append(mxv)
            round_att.append(int(res.stats[2]))
            if mxv < 0.01:
                break
        torch.cuda.synchronize()
        result["loop"] = {"rounds": rounds, "max_area_error": mxv,
                          "total_ms": round(1e3 * (time.perf_counter() - t_loop), 2),
                          "ms_per_round": round_ms, "max_error_per_round": round_err,
                          "attempts_per_round": round_att}
        # angular distortion of the final map, from the advected grid nodes
        d0, d1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ctx.distortion(pts[V:], per_square=True)            # first launch loads the kernels
        d0.record(stream)
        dst, _, _ = ctx.distortion(pts[V:], per_square=True)
        d1.record(stream)
        torch.cuda.synchronize()
        dst = dst.cpu().numpy()
        result["loop"]["distortion"] = {
            "e_a": float(dst[0]), "e_inf": float(dst[1]), "e_tilde_a": float(dst[2]),
            "e_tilde_inf": float(dst[3]), "folded_squares": int(dst[4]),
            "ms": round(d0.elapsed_time(d1), 4)}
        # inverse of the piecewise-linear map at a graticule sampled every
        # half cell of the cartogram box
        sq = torch.arange(0.25, L, 0.5, device=dev, dtype=torch.float32)
        gq = torch.stack(torch.meshgrid(sq, sq, indexing="xy"), -1).reshape(-1, 2).contiguous()
        ctx.inverse(pts[V:], gq)                              # warm-up (workspace)
        d0.record(stream)
        tri, pre = ctx.inverse(pts[V:], gq)
        d1.record(stream)
        torch.cuda.synchronize()
        ms_inv = d0.elapsed_time(d1)
        found = int((tri >= 0).sum())
        result["loop"]["inverse"] = {"queries": int(gq.shape[0]), "found": found,
                                     "ms": round(ms_inv, 4),
                                     "queries_per_s": round(gq.shape[0] / (ms_inv * 1e-3), 1)}

    if not args.no_diffusion:
        result["diffusion"] = diffusion_leg(args, dev, m, ctx, geom, value, pts0, pts, V,
                                            result.get("loop"))
    ctx.close()
    if not args.no_grad:
        result["grad"] = grad_leg(args, dev)
    if not args.no_batch:
        result["batch"] = batch_leg(args, dev)
    if not args.no_rect:
        result["rect"] = rect_leg(args, dev)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(m, pts_h, args)
    # the paper's own timings (context only: whole cartograms of real maps at
    # L = 512 on a 12-core Xeon E5-2680v3, divided by their round counts)
    result["paper_context"] = {
        "hardware": "Dell Precision T7810, 12-core Intel Xeon E5-2680v3 (multi-core C program with an FFT library)",
        "grid": "L = 512", "maps": "USA / India / China (real data, not available here)",
        "s_per_round": {"USA": round(1.5 / 5, 3), "India": round(2.6 / 12, 3),
                        "China": round(2.7 / 6, 3)},
        "note": "whole-run wall time / rounds, including set-up and I/O; different maps, "
                "grid size and hardware: context, not a target"}
    print(json.dumps(result), flush=True)


def diffusion_leg(args, dev, m, ctx, geom, value, pts0, pts, V, ffb_loop, max_rounds=30):
    """The comparison method of the paper on the same map and grid: the
    diffusion cartogram written as a flow-based projection (fields rebuilt
    at every stage time, integration to the cut-off time), rounds with the
    same blur schedule until max |e_r| < 1 %."""
    import torch
    import paper_1802_07625_amd as ffb

    opts = ffb.IntegrateOpts(tol=args.tol)
    pts.copy_(pts0)                                   # warm-up round (graph capture, buffers)
    ffb.iterate_diffusion(ctx, geom, value, pts, ffb.default_sigma(0), opts)
    torch.cuda.synchronize()
    # as in the FFB loop: sorted in round 0, that order kept for later rounds
    # (setting the option drops the order kept by the warm-up)
    ctx.set_option(ffb.OPT_POINT_ORDER, ffb.POINT_ORDER_KEEP)
    pts.copy_(pts0)
    torch.cuda.synchronize()
    area, errs, atts, round_ms = None, [], [], []
    t0 = time.perf_counter()
    for k in range(max_rounds):
        t_r = time.perf_counter()
        res = ffb.iterate_diffusion(ctx, geom, value, pts, ffb.default_sigma(k), opts,
                                    area_before=area)
        area = res.area_after
        mx = float(res.max_err_after)
        round_ms.append(round(1e3 * (time.perf_counter() - t_r), 3))
        errs.append(mx)
        atts.append(int(res.stats[2]))
        if mx < 0.01:
            break
    torch.cuda.synchronize()
    total = 1e3 * (time.perf_counter() - t0)
    dst, _, _ = ctx.distortion(pts[V:])
    dst = dst.cpu().numpy()
    out = {"rounds": len(errs), "max_area_error": errs[-1], "total_ms": round(total, 2),
           "ms_per_round": round_ms, "attempts_per_round": atts,
           "ms_per_attempt": round(total / max(1, sum(atts)), 4),
           "t_end": ffb.diffusion_t_end(m.lx, m.ly),
           "distortion": {"e_a": float(dst[0]), "e_inf": float(dst[1]),
                          "e_tilde_a": float(dst[2]), "e_tilde_inf": float(dst[3]),
                          "folded_squares": int(dst[4])}}
    if ffb_loop:
        out["ffb_loop_ms"] = ffb_loop["total_ms"]
        out["diffusion_over_ffb"] = round(total / ffb_loop["total_ms"], 3)
    return out


def rect_leg(args, dev, name="rect_1024x512", max_rounds=30):
    """The converging loop on a 1024 x 512 box whose regions include
    enclaves (host regions with clockwise hole rings) and multipolygons."""
    import torch
    import synth
    import paper_1802_07625_amd as ffb

    m = synth.workload(name)
    V = m.n_vertices
    pts_h = np.concatenate([m.xy, synth.grid_nodes(m.lx, m.ly)]).astype(np.float32)
    pts0 = torch.as_tensor(pts_h, device=dev)
    pts = pts0.clone()
    geom = ffb.Geometry.from_map(m, xy=pts[:V])
    value = torch.as_tensor(m.value, dtype=torch.float64, device=dev)
    ctx = ffb.Context(m.lx, m.ly, max_points=pts_h.shape[0])
    opts = ffb.IntegrateOpts(tol=args.tol)

    def loop():
        pts.copy_(pts0)
        area, out = None, []
        for k in range(max_rounds):
            res = ffb.iterate(ctx, geom, value, pts, ffb.default_sigma(k), opts, area_before=area)
            area = res.area_after
            mx = float(res.max_err_after)
            out.append(mx)
            if mx < 0.01:
                break
        return out

    loop()                                   # warm-up (kernel loading, allocations)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    errs = loop()
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    dst, _, _ = ctx.distortion(pts[V:])
    dst = dst.cpu().numpy()
    ctx.sync()
    ctx.close()
    holes = sum(1 for g in range(m.n_rings) if _signed_ring_area(m, g) < 0)
    return {"workload": name, "lx": m.lx, "ly": m.ly, "regions": m.n_regions,
            "rings": m.n_rings, "hole_rings": holes,
            "multi_ring_regions": int(np.sum(np.bincount(m.ring_region) > 1)),
            "vertices": V, "points": int(pts_h.shape[0]), "rounds": len(errs),
            "max_area_error": errs[-1], "total_ms": round(1e3 * total, 2),
            "distortion": {"e_a": float(dst[0]), "e_inf": float(dst[1]),
                           "e_tilde_a": float(dst[2]), "e_tilde_inf": float(dst[3]),
                           "folded_squares": int(dst[4])}}


def _signed_ring_area(m, g):
    p = m.xy[m.ring_vidx[m.ring_offsets[g]:m.ring_offsets[g + 1]]].astype(np.float64)
    return 0.5 * float(np.sum(p[:, 0] * np.roll(p[:, 1], -1) - np.roll(p[:, 0], -1) * p[:, 1]))


def batch_leg(args, dev, max_rounds=30):
    """The batched workload: maps c4_0 .. c4_{n-1} (L drawn from 128, 256,
    512; 20-200 regions; lognormal densities), every map iterated to max
    |e_r| < 1 % or 30 rounds.  Batched: one batch, launch shapes autotuned
    once, each round one graph replay for all active maps.  Baseline: the
    same maps one after another through the single-map entry points, one
    host read per round.  Both start from the resident input maps."""
    import torch
    import synth
    import paper_1802_07625_amd as ffb

    names = [f"c4_{i}" for i in range(args.batch_maps)]
    maps = [synth.workload(n) for n in names]
    opts = ffb.BatchOpts(max_rounds=max_rounds)

    def batched(ms):
        b = ffb.Batch(ms)
        pts0 = b.points.clone()
        shapes = b.autotune(opts)
        b.run(opts)                              # warm-up (graph capture)
        b.points.copy_(pts0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters = b.run(opts)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        rounds, mx, _, _ = b.results()
        b.close()
        return t, iters, rounds, mx, shapes

    t_batch, iters, rounds, mx, shapes = batched(maps)
    conv = [k for k in range(len(maps)) if mx[k] < 0.01]
    # the maps that stop below 1 % on their own, batched without the maps
    # that run to the round cap
    t_bconv, iters_conv, _, mx_conv, _ = batched([maps[k] for k in conv])

    # per-map loop, each map timed on its own
    ctxs = {}
    loop_rounds, loop_conv, t_maps = [], [], []
    dev_maps = []
    for m in maps:
        pts = torch.as_tensor(m.xy.astype(np.float32), device=dev)
        dev_maps.append((m, pts.clone(), pts, ffb.Geometry.from_map(m, xy=pts),
                         torch.as_tensor(m.value, dtype=torch.float64, device=dev)))
        key = (m.lx, m.ly)
        if key not in ctxs:
            ctxs[key] = ffb.Context(m.lx, m.ly, max_points=0)
    torch.cuda.synchronize()
    for m, p0, pts, geom, value in dev_maps:
        ctx = ctxs[(m.lx, m.ly)]
        area = None
        t0 = time.perf_counter()
        ok = False
        for k in range(max_rounds):
            res = ffb.iterate(ctx, geom, value, pts, ffb.default_sigma(k), area_before=area)
            area = res.area_after
            e = float(res.max_err_after)
            if e < 0.01:
                ok = True
                break
        t_maps.append(time.perf_counter() - t0)
        loop_conv.append(ok)
        loop_rounds.append(k + 1)
    for c in ctxs.values():
        c.close()
    t_loop = float(np.sum(t_maps))
    t_lconv = float(np.sum([t for t, ok in zip(t_maps, loop_conv) if ok]))
    n = len(maps)
    nc = len(conv)
    return {"workload": f"c4_0..c4_{n - 1}", "maps": n,
            "points": int(sum(m.n_vertices for m in maps)),
            "max_rounds": max_rounds, "stop": "max |e_r| < 1 %",
            "batched_ms": round(1e3 * t_batch, 2),
            "batched_maps_per_s": round(n / t_batch, 1),
            "batched_iterations": int(iters),
            "batched_converged": nc,
            "loop_ms": round(1e3 * t_loop, 2), "loop_maps_per_s": round(n / t_loop, 1),
            "loop_converged": int(np.sum(loop_conv)), "loop_rounds_total": int(sum(loop_rounds)),
            "batched_rounds_total": int(rounds.sum()),
            "speedup": round(t_loop / t_batch, 2),
            "note": "all maps: the maps still above 1 % after max_rounds count as done",
            "converged_only": {
                "maps": nc, "batched_ms": round(1e3 * t_bconv, 2),
                "batched_maps_per_s": round(nc / t_bconv, 1),
                "batched_iterations": int(iters_conv),
                "batched_still_converged": int(np.sum(mx_conv < 0.01)),
                "loop_ms": round(1e3 * t_lconv, 2), "loop_maps_per_s": round(nc / t_lconv, 1),
                "speedup": round(t_lconv / t_bconv, 2)},
            "capped": {"maps": n - nc, "rounds": max_rounds,
                       "final_max_error_range": [round(float(mx[k]), 4) for k in
                                                 (int(np.argmin(np.where(mx >= 0.01, mx, np.inf))),
                                                  int(np.argmax(mx)))] if n > nc else []},
            "shapes": shapes}


def _advect_sha():
    """Hash of the sources k_advect is compiled from (its file and the shared
    advection helpers): the counter figures above hold only for them."""
    import hashlib
    h = hashlib.sha256()
    for name in ("k_advect.hip", "advect_common.h"):
        with open(os.path.join(ROOT, "paper_1802_07625_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def grad_leg(args, dev, workload="c5_L512", rounds=3, max_steps=256):
    """fwd = `rounds` FFB rounds (areas, density, flux, integration, areas);
    fwd+bwd = the same rounds recorded on the tape plus ffb_backward for
    dL/d(value) of a loss of the final areas.  Both start from the same
    resident map; times are per whole run, averaged over --grad-steps."""
    import torch
    import synth
    import paper_1802_07625_amd as ffb

    m = synth.workload(workload)
    L, V = m.lx, m.n_vertices
    sigmas = [ffb.default_sigma(k) for k in range(rounds)]
    out = {"workload": workload, "rounds": rounds, "sigmas": sigmas, "regions": m.n_regions,
           "vertices": V}
    for label, with_grid in (("", True), ("_vertices_only", False)):
        parts = [m.xy.astype(np.float32)]
        if with_grid:
            parts.append(synth.grid_nodes(L, L))
        pts0 = torch.as_tensor(np.concatenate(parts), device=dev)
        pts = pts0.clone()
        ctx = ffb.Context(L, L, max_points=pts.shape[0])
        geom = ffb.Geometry.from_map(m, xy=pts[:V])
        value = torch.as_tensor(m.value, dtype=torch.float64, device=dev)
        g_area = torch.ones(m.n_regions, dtype=torch.float64, device=dev)

        def fwd():
            pts.copy_(pts0)
            area, _, _ = ctx.area_error(geom, value)
            for s in sigmas:
                rho, _ = ctx.density(geom, value, area)
                f, rb = ctx.flux(rho, s)
                ctx.integrate(f, rb, pts, h_cap=0)
                area, _, _ = ctx.area_error(geom, value)

        def fwd_bwd():
            pts.copy_(pts0)
            ffb.FFBFunction.apply(value, ctx, geom, pts, sigmas, None, max_steps, None)
            ctx.backward(g_area)

        times = {}
        for name, fn in (("fwd", fwd), ("fwd_bwd", fwd_bwd)):
            for _ in range(2):
                fn()
            ctx.sync()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.grad_steps):
                fn()
            torch.cuda.synchronize()
            times[name] = 1e3 * (time.perf_counter() - t0) / args.grad_steps
        ctx.sync()
        ctx.close()
        if with_grid:
            out["points"] = int(pts0.shape[0])
        out["fwd_ms" + label] = round(times["fwd"], 4)
        out["fwd_bwd_ms" + label] = round(times["fwd_bwd"], 4)
        out["ratio" + label] = round(times["fwd_bwd"] / times["fwd"], 3)
    # the C5 configuration advects only the polygon vertices (grid nodes do
    # not enter the loss); the run with all grid nodes is reported beside it
    out["c5_ratio"] = out["ratio_vertices_only"]
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(m, pts_h, args):
    """The FP64 oracle, untuned, on the host cores: whole iterations of the
    same workload (areas, raster, direct-sum transforms, advection of every
    vertex and grid node with the oracle's own step control, areas), repeated
    until about ten seconds of work have been timed; then the same phases on
    one core, the advection on a 1/32 sample of the points with the step
    schedule of the all-core run replayed (its cost is proportional to the
    number of points), scaled to the whole iteration."""
    import oracle
    cores = oracle.set_threads(0)
    runs, t = [], {}
    while sum(runs) < args.cpu_seconds or not runs:
        t0 = time.perf_counter()
        a = oracle.region_areas(m)
        t["area"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        rho, _ = oracle.density(m, m.value, a)
        t["density"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        F = oracle.flux(rho, args.sigma)
        t["flux"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        r = oracle.integrate(F, pts_h.astype(np.float64), oracle.IntegrateOpts(tol=args.tol))
        t["advect"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.region_areas(m, r.xy[:m.n_vertices])
        t["area_after"] = time.perf_counter() - t0
        runs.append(sum(t.values()))
    out = {"value": round(1e3 * float(np.mean(runs)), 1), "unit": "ms/iteration",
           "cores": cores, "kind": "oracle", "cpu_model": _cpu_model(),
           "sample": (f"{len(runs)} whole iterations of the same workload at full size "
                      f"({pts_h.shape[0]} points; the oracle's own step control took "
                      f"{r.accepted} accepted and {r.rejected} rejected steps)"),
           "phases_s": {k: round(v, 3) for k, v in t.items()}}
    if args.cpu_single:
        oracle.set_threads(1)
        one = {}
        t0 = time.perf_counter()
        a = oracle.region_areas(m)
        one["area"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        rho, _ = oracle.density(m, m.value, a)
        one["density"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        F = oracle.flux(rho, args.sigma)
        one["flux"] = time.perf_counter() - t0
        sub = pts_h[::32].astype(np.float64)
        t0 = time.perf_counter()
        oracle.integrate(F, sub, oracle.IntegrateOpts(tol=args.tol), replay_h=r.h)
        one["advect"] = (time.perf_counter() - t0) * pts_h.shape[0] / sub.shape[0]
        one["area_after"] = one["area"]
        oracle.set_threads(0)
        out["single_core"] = {
            "value": round(1e3 * sum(one.values()), 1), "unit": "ms/iteration", "cores": 1,
            "sample": (f"areas, raster and transforms once at full size; advection of every "
                       f"32nd point ({sub.shape[0]}) with the {len(r.h)} accepted steps of the "
                       f"all-core run replayed, scaled by {pts_h.shape[0] / sub.shape[0]:.2f}"),
            "phases_s": {k: round(v, 3) for k, v in one.items()}}
    return out


if __name__ == "__main__":
    main()
