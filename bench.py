#!/usr/bin/env python3
"""Throughput of the direction-fusion hot path on one MI355X.

One step = one pass of the whole path over one batch of synthetic input with
every input already resident in HBM.  Prints ONE JSON line on stdout (logs go
to stderr).  Only one GPU is used; --gpus above 1 exits with a message.

Workloads (synthetic scenes from ``scenegen``; they stand in for the paper's
rendered Hair20K hairstyles and captured videos, which are not available).
Points lie on the visible outer layer of the hair and every form applies the
depth visibility test of Sec. 3.1.1 with the scene's rendered depth maps
(--no-depth switches it off):
  metric     (default) 8 heads x 250k points of tight curls, 128 views at
             1024^2 float16, kappa 10, 30% outliers: learned+batched (value)
             against plain per head, plus plain+batched and learned per head.
  plain      500k points on 20k straight/wavy strands, 64 views at 1024^2
             float16 maps, 10% outlier texels, 5x5 patch, 128 candidates +
             8 refinement iterations (fd_fuse_directions, plain mode).
  learned    the same scene, learned form against plain.
  batched    16 uneven hairstyles (50k-800k points, 32-128 views, 512-1024
             px float16 maps): plain search of all in one captured batched
             launch against one call per scene.
  gabor      orientation and confidence maps from 64 grey frames at 1024^2
             (the plain workload's views; 32 orientations, radius 8), then
             the plain search of the plain workload on those maps.
  volume     occupancy / orientation volume of 2M oriented points over the
             realistic hairstyle's volume (10 deg direction noise, 10%
             outliers) on a 2 mm grid.
  train      proposal-network training (112 -> 256 -> 256 -> 256 -> 3, BF16
             MFMA): Adam steps of batch 4096 on the features and plain-search
             directions of the realistic scene's 500k points.
  pipeline   the chain on one GPU: 64 grey frames at 1024^2 -> orientation
             maps -> plain direction search of the 500k outer points ->
             volume of those points and 1.5M inner stand-in points (3 mm)
             -> hair growing, linking and strand assembly.
  phg        parallel hair growing through the volume of 8M such points on
             a 3 mm grid: 20k guide strands from the scalp roots (batches of
             4096, deferred occupancy), interior segments from every third
             voxel traced both ways, the Eq. 13 linking of all pieces and
             the assembly of the linked pieces into strands.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fused points/s at ≤2° mean angular err; learned+batched vs plain, 1 MI355X"
PEAK_FP32 = 157.3             # TFLOP/s: MI355X published fp32 vector peak
PEAK_FP32_MFMA = 157.3        # TFLOP/s: dense fp32 matrix-core figure (v_mfma_f32_*_f32)
PEAK_HBM = 8000.0             # GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# HBM bytes per launch of the search kernels, from rocprofv3 --pmc FETCH_SIZE
# and WRITE_SIZE passes (summaries under profiles/), each scaled by what the
# same counter reads for a 512 MiB device copy (FETCH_SIZE x 2, WRITE_SIZE
# x 1).  A figure holds only for the kernel sources it was taken with: `src`
# is a hash of them, and a changed source reports null.
_SEARCH_SOURCES = ["fd_search.hpp", "fd_fuse.hip", "fd_device.hpp", "fd_kernels.hpp"]
_BATCHED_SOURCES = _SEARCH_SOURCES + ["fd_batched.hip"]
_GABOR_SOURCES = ["fd_gabor.hip"]
_VOLUME_SOURCES = ["fd_volume.hip", "fd_voxel.hpp"]
_PHG_SOURCES = ["fd_phg.hip", "fd_voxel.hpp"]
TRAFFIC = {
    "k_fuse, realistic 500k": {"read": 409.9e6, "write": 37.6e6, "files": _SEARCH_SOURCES,
                               "src": "f1cf612e32964315"},
    "k_fuse, metric workload, per head": {"read": 135.8e6, "write": 8.5e6,
                                          "files": _SEARCH_SOURCES, "src": "f1cf612e32964315"},
    "k_b_learned, metric workload": {"read": 2258.3e6, "write": 160.7e6,
                                     "files": _BATCHED_SOURCES, "src": "b9fe1b77b1dd8781"},
    # the autotuned one-wave-per-tile form (the persistent form's traffic
    # depends on its queue shape)
    "k_b_fuse_tiles, 16 hairstyles": {"read": 3812.9e6, "write": 348.6e6,
                                      "files": _BATCHED_SOURCES, "src": "b9fe1b77b1dd8781"},
    "k_gabor_mfma, 64 frames 1024^2": {"read": 1152.1e6, "write": 406.8e6,
                                       "files": _GABOR_SOURCES, "src": "21a8f3739c8a0866"},
    # the counting sort: keys and counts, the scan, the placement
    "volume sort, realistic 2M points 2 mm": {"read": 319.8e6, "write": 237.4e6,
                                              "files": _VOLUME_SOURCES,
                                              "src": "b0b5904bb1ae7e7b"},
    # per pass: the 5 guide batches and the 2 segment launches
    "k_grow, phg workload": {"read": 201.9e6, "write": 30.7e6, "files": _PHG_SOURCES,
                             "src": "4f42252c325b0cf8"},
}


def _src_hash(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2604_05794_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_of(key):
    t = TRAFFIC.get(key)
    if t is None or _src_hash(t["files"]) != t["src"]:
        return None
    return t["read"] + t["write"]


# One sim-eval is one (direction, view, patch sample) evaluation of the
# objective; it is counted as 6 flop (the sample's share of the direction's
# image vector and doubled angle plus its quadratic form), as in the
# roofline accounting of the search.
FLOP_PER_SIM_EVAL = 6


def sim_evals_full(patch, n_cand, iters, top_k=5):
    """Sim-evals of one plain search: lattice plus six stencil directions per
    refinement iteration, in each of the top_k views, at every patch
    sample."""
    return (n_cand + 6 * iters) * top_k * patch * patch


def sim_evals_refine(patch, iters, top_k=5):
    """Sim-evals of the learned form's short refinement from a proposal."""
    return (1 + 6 * iters) * top_k * patch * patch


def plain_flop_per_point(patch, n_cand, iters, top_k=5):
    return FLOP_PER_SIM_EVAL * sim_evals_full(patch, n_cand, iters, top_k)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sc, kw, seconds, depth=True):
    """The oracle, untuned, on a bounded sample of the same scene: points in
    stride order (stride 7919, modulo N, wrapping around) until `seconds`
    have passed, on every host thread; then the same on one thread for a
    third of that time."""
    import numpy as np
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    threads = min(threads, os.cpu_count() or threads)
    orc = oracle.Oracle(sc.cams, sc.theta, sc.conf, depth=sc.depth if depth else None, **kw)
    n = sc.n_points
    stride = 7919

    def run(nthr, secs):
        chunk = 64 * nthr
        done = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < secs:
            idx = (np.arange(done, done + chunk) * stride) % n
            orc.fuse(sc.points[idx], n_threads=nthr)
            done += chunk
        return done, time.perf_counter() - t0

    done, el = run(threads, seconds)
    done1, el1 = run(1, seconds / 3.0)
    return {"value": done / el, "unit": "points/s", "cores": threads, "kind": "oracle",
            "cpu_model": _cpu_model(), "logical_cpus": os.cpu_count(),
            "sample": f"{done} points of the same scene ({n} points; stride {stride} modulo N), "
                      f"{el:.1f} s, binary64 oracle, OpenMP over points",
            "single_thread": {"value": done1 / el1, "unit": "points/s", "cores": 1,
                              "sample": f"{done1} points, {el1:.1f} s, same order"}}


def _axial_deg(a, b):
    import torch
    c = torch.linalg.norm(torch.cross(a, b, dim=1), dim=1)
    d = torch.abs((a * b).sum(1))
    return torch.rad2deg(torch.atan2(c, d))


def _stage_times(ctx, stages_list):
    stages = {}
    for nm, st in stages_list:
        ms, cnt = ctx.stage_time(st)
        if cnt:
            stages[nm] = ms / cnt
    return stages


def _timed(step, args, ctx, stages_list, profile=True):
    """Wall time of args.steps steps after args.warmup; with profile, the
    per-stage kernel times (HIP events on the launch stream) of the timed
    steps."""
    import torch
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile(profile)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    stages = _stage_times(ctx, stages_list) if profile else {}
    ctx.profile(False)
    return el, stages


def _stage_pass(step, ctx, stages_list, reps=3):
    """Per-stage kernel times of `reps` extra steps run with stage timing on
    (the batched form then launches its kernels directly rather than from
    its graph, so that HIP events can sit between its stages)."""
    import torch
    torch.cuda.synchronize()
    ctx.profile(True)
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    stages = _stage_times(ctx, stages_list)
    ctx.profile(False)
    return stages


def run_learned(args):
    """Learned form on the realistic scene: network proposal, 2 refinement
    iterations, plain search where the refined cost exceeds the calibrated
    threshold.  Compared with the plain search on the same scene."""
    import numpy as np
    import torch
    import scenegen
    from paper_2604_05794_amd import native

    name = "realistic"
    rec = scenegen.RECIPES[name]
    kw = dict(patch=rec["patch"], n_candidates=rec["n_candidates"],
              refine_iters=rec["refine_iters"], top_k=5)
    t = time.perf_counter()
    sc = scenegen.make_scene(name, args.seed)
    log(f"generated {name}: {sc.n_points} points in {time.perf_counter() - t:.1f} s")
    dev = torch.device("cuda:0")
    pts = torch.from_numpy(sc.points).to(dev)
    cams = torch.from_numpy(sc.cams).to(dev)
    th = torch.from_numpy(sc.theta).to(dev)
    cf = torch.from_numpy(sc.conf).to(dev)
    gt = torch.from_numpy(sc.gt).to(dev)
    if not args.no_depth:
        kw["depth_maps"] = torch.from_numpy(sc.depth).to(dev)
    n = sc.n_points
    ctx = native.Context(max_points=n)
    net = native.MLP(path=args.mlp)
    step0, tau = net.calibration()
    log(f"network {args.mlp}: learned_step0 {step0:.4f} rad, fallback_cost {tau:.4f}")
    stream = torch.cuda.current_stream()
    dp = torch.empty((n, 3), dtype=torch.float32, device=dev)
    cp = torch.empty((n,), dtype=torch.float32, device=dev)
    dl = torch.empty_like(dp)
    cl = torch.empty_like(cp)
    stg = [("tiling", native.FD_STAGE_TILING), ("topk", native.FD_STAGE_TOPK),
           ("fuse", native.FD_STAGE_FUSE), ("features", native.FD_STAGE_FEATURES),
           ("mlp", native.FD_STAGE_MLP), ("refine", native.FD_STAGE_REFINE),
           ("fallback", native.FD_STAGE_FALLBACK)]

    def plain():
        native.fuse_directions(pts, cams, th, cf, dirs=dp, costs=cp, ctx=ctx, stream=stream, **kw)

    def learned():
        native.fuse_directions(pts, cams, th, cf, dirs=dl, costs=cl, ctx=ctx, stream=stream,
                               mode=native.FD_MODE_LEARNED, mlp=net, learned_iters=2,
                               learned_step0=step0, fallback_cost=tau,
                               head_centre=sc.head_centre, **kw)

    el_p, st_p = _timed(plain, args, ctx, stg)
    el_l, st_l = _timed(learned, args, ctx, stg)
    n_fb = ctx.fallback_count()
    fin = torch.isfinite(cp)
    err = _axial_deg(dl[fin], dp[fin])
    err_gt_l = _axial_deg(dl[fin], gt[fin])
    err_gt_p = _axial_deg(dp[fin], gt[fin])
    v_p = n / (el_p / args.steps)
    v_l = n / (el_l / args.steps)
    log(f"plain {v_p / 1e6:.1f} M points/s {json.dumps({k: round(v, 4) for k, v in st_p.items()})}")
    log(f"learned {v_l / 1e6:.1f} M points/s {json.dumps({k: round(v, 4) for k, v in st_l.items()})}"
        f" fallback {n_fb / n:.4f}, mean err vs plain {float(err.mean()):.3f} deg")
    kw.pop("depth_maps", None)
    flop = plain_flop_per_point(kw["patch"], kw["n_candidates"], kw["refine_iters"], 5)
    achieved = flop * n / (st_p["fuse"] * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": v_l, "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el_l * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "learned (unbatched): 500k points, 64 views 1024^2 f16, 10% "
                               "outliers, P=5; network proposal + 2 refinement iterations, "
                               "plain fallback (128 candidates + 8 iterations)",
                   "mode": "learned", "points": n, "views": sc.n_views,
                   "depth_test": not args.no_depth, **kw},
        "plain_points_per_s": v_p, "speedup_vs_plain": v_l / v_p,
        "mean_err_vs_plain_deg": float(err.mean()),
        "median_err_vs_plain_deg": float(err.median()),
        "mean_err_vs_gt_deg": {"learned": float(err_gt_l.mean()), "plain": float(err_gt_p.mean())},
        "fallback_frac": n_fb / n,
        "stages_ms_per_launch": {"plain": st_p, "learned": st_l},
        "roofline": {"bound": "alu", "kernel": "k_fuse", "achieved": achieved,
                     "peak": PEAK_FP32, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32,
                     "traffic": traffic_of("k_fuse, realistic 500k"),
                     "avg_launch_ms": st_p["fuse"], "flop_per_point": flop},
    }
    return out


def run_metric(args):
    """The hard set: 8 heads of tight curls (250k points each, 128 views at
    1024^2 float16, kappa 10, 30% outlier texels).  Plain = fd_fuse_directions
    per head; learned+batched = the network proposal, 2 refinement iterations
    and the plain search where the refined cost exceeds the calibrated
    threshold, for all 8 heads in one captured batched launch.  Also times
    plain+batched and learned per head, and reports the learned result's
    angle to the plain one."""
    import numpy as np
    import torch
    import scenegen
    from paper_2604_05794_amd import native

    rec = scenegen.RECIPES["curls"]
    kw = dict(patch=rec["patch"], n_candidates=rec["n_candidates"],
              refine_iters=rec["refine_iters"], top_k=5)
    dev = torch.device("cuda:0")
    heads = []
    t = time.perf_counter()
    for h in range(args.heads):
        sc = scenegen.make_scene("curls", args.seed + h)
        d = dict(points=torch.from_numpy(sc.points).to(dev),
                 cams=torch.from_numpy(sc.cams).to(dev),
                 orient_maps=torch.from_numpy(sc.theta).to(dev),
                 conf_maps=torch.from_numpy(sc.conf).to(dev),
                 dirs=torch.empty((sc.n_points, 3), dtype=torch.float32, device=dev),
                 costs=torch.empty((sc.n_points,), dtype=torch.float32, device=dev),
                 head_centre=sc.head_centre, gt=torch.from_numpy(sc.gt).to(dev))
        if not args.no_depth:
            d["depth_maps"] = torch.from_numpy(sc.depth).to(dev)
        heads.append((sc, d))
        log(f"head {h}: {sc.n_points} points, {sc.n_views} views "
            f"({time.perf_counter() - t:.1f} s)")
    n = sum(sc.n_points for sc, _ in heads)
    stream = torch.cuda.current_stream()
    ctx = native.Context(max_points=n, max_views=sum(sc.n_views for sc, _ in heads),
                         max_scenes=len(heads))
    net = native.MLP(path=args.mlp)
    step0, tau = net.calibration()
    lkw = dict(mode=native.FD_MODE_LEARNED, mlp=net, learned_iters=2, learned_step0=step0,
               fallback_cost=tau)
    outs = {}
    stg = [("tiling", native.FD_STAGE_TILING), ("topk", native.FD_STAGE_TOPK),
           ("fuse", native.FD_STAGE_FUSE), ("features", native.FD_STAGE_FEATURES),
           ("mlp", native.FD_STAGE_MLP), ("refine", native.FD_STAGE_REFINE),
           ("fallback", native.FD_STAGE_FALLBACK), ("batched", native.FD_STAGE_BATCHED)]

    def per_head(extra):
        def step():
            for sc, d in heads:
                native.fuse_directions(d["points"], d["cams"], d["orient_maps"], d["conf_maps"],
                                       dirs=d["dirs"], costs=d["costs"], ctx=ctx, stream=stream,
                                       head_centre=sc.head_centre,
                                       depth_maps=d.get("depth_maps"), **kw, **extra)
        return step

    def batched(extra):
        scenes = [d for _, d in heads]

        def step():
            native.fuse_batched(scenes, ctx, stream=stream, **kw, **extra)
        return step

    # tile shapes of each batched form, picked by the autotuner (untimed):
    # persistent tile queues or one wave per tile
    tuned = {}
    for name, extra in (("plain_batched", {}), ("learned_batched", lkw)):
        t = time.perf_counter()
        native.autotune([d for _, d in heads], ctx, stream=stream, **kw, **extra)
        tuned[name] = ctx.tuned()
        log(f"autotune {name}: {time.perf_counter() - t:.1f} s, chunk {tuned[name][0]}, "
            f"grid {tuned[name][1]}")

    def snap():
        return (torch.cat([d["dirs"] for _, d in heads]).clone(),
                torch.cat([d["costs"] for _, d in heads]).clone())

    res = {}
    n_fb_batched = None
    for name, fn in (("plain", per_head({})), ("plain_batched", batched({})),
                     ("learned", per_head(lkw)), ("learned_batched", batched(lkw))):
        is_batched = name.endswith("batched")
        if is_batched:
            ctx.set_tuned(*tuned[name])
        # every form is timed with stage timing off; the stage times come
        # from a separate pass (the batched forms then launch the same
        # kernels directly instead of replaying their graph)
        el, _ = _timed(fn, args, ctx, stg, profile=False)
        outs[name] = snap()
        st = _stage_pass(fn, ctx, stg)
        if name == "learned_batched":
            fb_listed, fb_inplace = ctx.fallback_split(stream)
            n_fb_batched = fb_listed + fb_inplace
        res[name] = (n / (el / args.steps), el * 1e3 / args.steps, st)
        log(f"{name}: {res[name][0] / 1e6:.1f} M points/s, {res[name][1]:.3f} ms/step, "
            f"{json.dumps({k: round(v, 4) for k, v in st.items()})}")
    dp, cp = outs["plain"]
    fin = torch.isfinite(cp)
    gt = torch.cat([d["gt"] for _, d in heads])
    errs = {k: float(_axial_deg(outs[k][0][fin], dp[fin]).mean()) for k in outs}
    err_gt = {k: float(_axial_deg(outs[k][0][fin], gt[fin]).mean()) for k in outs}
    same_pb = bool(torch.equal(outs["plain_batched"][0], dp))
    same_lb = bool(torch.equal(outs["learned_batched"][0], outs["learned"][0]))
    # fallback share of the learned form (per-head calls leave the last head's count)
    ctx.profile(False)
    fb = 0
    for sc, d in heads:
        native.fuse_directions(d["points"], d["cams"], d["orient_maps"], d["conf_maps"],
                               dirs=d["dirs"], costs=d["costs"], ctx=ctx, stream=stream,
                               head_centre=sc.head_centre, depth_maps=d.get("depth_maps"),
                               **kw, **lkw)
        fb += ctx.fallback_count(stream)
    log(f"learned+batched fallback {n_fb_batched} of {n} points; "
        f"mean err vs plain (deg) {json.dumps({k: round(v, 3) for k, v in errs.items()})}; "
        f"fallback {fb / n:.3f}; batched == per-head: plain {same_pb}, learned {same_lb}")
    v_lb, ms_lb, st_lb = res["learned_batched"]
    v_p, _, st_p = res["plain"]
    flop = plain_flop_per_point(kw["patch"], kw["n_candidates"], kw["refine_iters"], 5)
    # dominant kernel of the learned+batched step: k_b_learned, which refines
    # every point from its proposal (1 + 6 x 2 directions) and runs the full
    # search in place for the waves that mostly fall back
    flop_refine = FLOP_PER_SIM_EVAL * sim_evals_refine(kw["patch"], lkw["learned_iters"])
    flop_lb = flop_refine * n + flop * fb_inplace
    achieved = flop_lb / (st_lb["refine"] * 1e-3) / 1e12
    achieved_plain = flop * n / (st_p["fuse"] * len(heads) * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": v_lb, "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_lb,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"learned+batched on hard data: {len(heads)} heads x 250k points "
                               "of tight curls (r 2-6 mm, pitch 4-10 mm), 128 views 1024^2 f16, "
                               "kappa 10, 30% outlier texels, P=5, 2 refinement iterations after "
                               "the network proposal, plain fallback (128 candidates + 8 "
                               "iterations), one captured batched launch",
                   "mode": "learned+batched", "points": n, "heads": len(heads), "views": 128,
                   "depth_test": not args.no_depth,
                   "learned_step0": step0, "fallback_cost": tau,
                   "batched_shape": {k: dict(zip(("chunk", "grid"), v)) for k, v in tuned.items()},
                   **kw},
        "plain_points_per_s": v_p, "speedup_vs_plain": v_lb / v_p,
        "points_per_s": {k: v[0] for k, v in res.items()},
        "ms_per_step_by_form": {k: v[1] for k, v in res.items()},
        "mean_err_vs_plain_deg": errs, "mean_err_vs_gt_deg": err_gt,
        "median_err_vs_gt_deg_plain": float(_axial_deg(dp[fin], gt[fin]).median()),
        "fallback_frac": fb / n, "batched_bitwise_equal": {"plain": same_pb, "learned": same_lb},
        "stages_ms_per_launch_plain": st_p,
        "roofline": {"bound": "alu",
                     "kernel": "k_b_learned: refinement "
                               "from the proposal for every point, full search in place for "
                               "the waves that mostly fall back (learned+batched step)",
                     "achieved": achieved, "peak": PEAK_FP32, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32,
                     "traffic": traffic_of("k_b_learned, metric workload"),
                     "avg_launch_ms": st_lb["refine"], "points_per_launch": n,
                     "full_searches_in_place": fb_inplace, "listed_fallbacks": fb_listed,
                     "flop_per_launch": flop_lb, "flop_per_full_search": flop,
                     "flop_per_refinement": flop_refine,
                     "flop_per_sim_eval": FLOP_PER_SIM_EVAL},
        "roofline_plain_per_head": {
            "bound": "alu", "kernel": "k_fuse (plain search, one launch per head)",
            "achieved": achieved_plain, "peak": PEAK_FP32, "unit": "TFLOP/s",
            "frac": achieved_plain / PEAK_FP32, "avg_launch_ms": st_p["fuse"],
            "points_per_launch": n // len(heads),
            "traffic": traffic_of("k_fuse, metric workload, per head")},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(heads[0][0], kw, args.cpu_seconds,
                                           depth=not args.no_depth)
        log(f"cpu baseline: {out['cpu_baseline']}")
    return out


def run_batched(args):
    """The uneven 16-hairstyle set (scene i: round(50k 16^(i/15)) points,
    32 + 32 (5i mod 4) views, [512, 768, 1024][7i mod 3] px float16 maps,
    the realistic recipe otherwise), plain search of all 16 scenes in one
    captured batched launch with the autotuned tile shape (value), against
    one fd_fuse_directions call per scene."""
    import torch
    import scenegen
    from paper_2604_05794_amd import native

    rec = scenegen.RECIPES["realistic"]
    kw = dict(patch=rec["patch"], n_candidates=rec["n_candidates"],
              refine_iters=rec["refine_iters"], top_k=5)
    dev = torch.device("cuda:0")
    scenes = []
    t = time.perf_counter()
    for i, r in enumerate(scenegen.batched_recipes(16)):
        sc = scenegen.make_scene(r, args.seed + i)
        d = dict(points=torch.from_numpy(sc.points).to(dev),
                 cams=torch.from_numpy(sc.cams).to(dev),
                 orient_maps=torch.from_numpy(sc.theta).to(dev),
                 conf_maps=torch.from_numpy(sc.conf).to(dev),
                 dirs=torch.empty((sc.n_points, 3), dtype=torch.float32, device=dev),
                 costs=torch.empty((sc.n_points,), dtype=torch.float32, device=dev))
        if not args.no_depth:
            d["depth_maps"] = torch.from_numpy(sc.depth).to(dev)
        scenes.append((sc, d))
        log(f"scene {i}: {sc.n_points} points, {sc.n_views} views {sc.width}^2 "
            f"({time.perf_counter() - t:.1f} s)")
    n = sum(sc.n_points for sc, _ in scenes)
    stream = torch.cuda.current_stream()
    ctx = native.Context(max_points=n, max_views=sum(sc.n_views for sc, _ in scenes),
                         max_scenes=len(scenes))
    devs = [d for _, d in scenes]
    stg = [("tiling", native.FD_STAGE_TILING), ("topk", native.FD_STAGE_TOPK),
           ("fuse", native.FD_STAGE_FUSE), ("batched", native.FD_STAGE_BATCHED)]

    def per_scene():
        for sc, d in scenes:
            native.fuse_directions(d["points"], d["cams"], d["orient_maps"], d["conf_maps"],
                                   dirs=d["dirs"], costs=d["costs"], ctx=ctx, stream=stream,
                                   depth_maps=d.get("depth_maps"), **kw)

    def batched():
        native.fuse_batched(devs, ctx, stream=stream, **kw)

    t = time.perf_counter()
    native.autotune(devs, ctx, stream=stream, **kw)
    tuned = ctx.tuned()
    log(f"autotune: {time.perf_counter() - t:.1f} s, chunk {tuned[0]}, grid {tuned[1]}")

    def snap():
        return (torch.cat([d["dirs"] for d in devs]).clone(),
                torch.cat([d["costs"] for d in devs]).clone())

    el_p, _ = _timed(per_scene, args, ctx, stg, profile=False)
    out_p = snap()
    st_p = _stage_pass(per_scene, ctx, stg)
    ctx.set_tuned(*tuned)
    el_b, _ = _timed(batched, args, ctx, stg, profile=False)
    out_b = snap()
    st_b = _stage_pass(batched, ctx, stg)
    same = bool(torch.equal(out_p[0], out_b[0]) and torch.equal(out_p[1], out_b[1]))
    v_b = n / (el_b / args.steps)
    v_p = n / (el_p / args.steps)
    log(f"batched: {v_b / 1e6:.1f} M points/s ({el_b * 1e3 / args.steps:.3f} ms/step) "
        f"{json.dumps({k: round(v, 4) for k, v in st_b.items()})}; per scene: "
        f"{v_p / 1e6:.1f} M points/s {json.dumps({k: round(v, 4) for k, v in st_p.items()})}; "
        f"bitwise equal {same}")
    flop = plain_flop_per_point(kw["patch"], kw["n_candidates"], kw["refine_iters"], 5)
    achieved = flop * n / (st_b["fuse"] * 1e-3) / 1e12
    kern = "k_b_fuse (persistent tile queue)" if tuned[1] > 0 else \
        "k_b_fuse_tiles (one wave per tile)"
    traffic_key = ("k_b_fuse" if tuned[1] > 0 else "k_b_fuse_tiles") + ", 16 hairstyles"
    out = {
        "metric": METRIC, "value": v_b, "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el_b * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched plain: 16 uneven hairstyles, {n} points in all "
                               "(50k-800k per scene), 32-128 views, 512-1024 px f16 maps, "
                               "realistic recipe, P=5, 128 candidates + 8 refinement "
                               "iterations, one captured batched launch",
                   "mode": "plain+batched", "points": n,
                   "scenes": [[sc.n_points, sc.n_views, sc.width] for sc, _ in scenes],
                   "depth_test": not args.no_depth,
                   "batched_shape": dict(zip(("chunk", "grid"), tuned)), **kw},
        "per_scene_points_per_s": v_p, "speedup_vs_per_scene": v_b / v_p,
        "ms_per_step_per_scene": el_p * 1e3 / args.steps,
        "batched_bitwise_equal_per_scene": same,
        "stages_ms_per_launch": st_b, "stages_ms_per_launch_per_scene": st_p,
        "roofline": {"bound": "alu", "kernel": kern, "achieved": achieved,
                     "peak": PEAK_FP32, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32,
                     "traffic": traffic_of(traffic_key), "avg_launch_ms": st_b["fuse"],
                     "points_per_launch": n, "flop_per_point": flop,
                     "flop_per_sim_eval": FLOP_PER_SIM_EVAL},
    }
    if not args.no_cpu_baseline:
        sc = scenes[len(scenes) // 2][0]
        out["cpu_baseline"] = cpu_baseline(sc, kw, args.cpu_seconds, depth=not args.no_depth)
        out["cpu_baseline"]["sample"] += f" (scene {len(scenes) // 2} of the set)"
    return out


def run_plain(args):
    import numpy as np
    import torch
    import scenegen
    from paper_2604_05794_amd import native

    name = "realistic"
    rec = scenegen.RECIPES[name]
    kw = dict(patch=rec["patch"], n_candidates=rec["n_candidates"],
              refine_iters=rec["refine_iters"], top_k=5)
    t = time.perf_counter()
    sc = scenegen.make_scene(name, args.seed)
    log(f"generated {name}: {sc.n_points} points, {sc.n_views} views {sc.width}x{sc.height} "
        f"{sc.theta.dtype} in {time.perf_counter() - t:.1f} s")
    dev = torch.device("cuda:0")
    pts = torch.from_numpy(sc.points).to(dev)
    cams = torch.from_numpy(sc.cams).to(dev)
    th = torch.from_numpy(sc.theta).to(dev)
    cf = torch.from_numpy(sc.conf).to(dev)
    dirs = torch.empty((sc.n_points, 3), dtype=torch.float32, device=dev)
    costs = torch.empty((sc.n_points,), dtype=torch.float32, device=dev)
    ctx = native.Context(max_points=sc.n_points)
    stream = torch.cuda.current_stream()
    dm = None if args.no_depth else torch.from_numpy(sc.depth).to(dev)

    def step():
        native.fuse_directions(pts, cams, th, cf, dirs=dirs, costs=costs, ctx=ctx,
                               stream=stream, depth_maps=dm, **kw)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    stages = {}
    for nm, st in (("tiling", native.FD_STAGE_TILING), ("topk", native.FD_STAGE_TOPK),
                   ("fuse", native.FD_STAGE_FUSE)):
        ms, cnt = ctx.stage_time(st)
        stages[nm] = ms / max(cnt, 1)
    ctx.profile(False)
    ms_step = el * 1e3 / args.steps
    value = sc.n_points / (el / args.steps)
    flop = plain_flop_per_point(kw["patch"], kw["n_candidates"], kw["refine_iters"], 5)
    fuse_s = stages["fuse"] * 1e-3
    achieved = flop * sc.n_points / fuse_s / 1e12
    c = costs.cpu().numpy()
    fin = torch.isfinite(costs)
    gt = torch.from_numpy(sc.gt).to(dev)
    err_gt = _axial_deg(dirs[fin], gt[fin])
    fpmvo = None
    if dm is not None:
        # the paper's own candidates (Eqs. 1-7) on the same scene, for comparison
        fd = torch.empty_like(dirs)
        fc = torch.empty_like(costs)

        def step_fp():
            native.fuse_directions(pts, cams, th, cf, dirs=fd, costs=fc, ctx=ctx, stream=stream,
                                   depth_maps=dm, mode=native.FD_MODE_FPMVO, **kw)
        el_f, st_f = _timed(step_fp, args, ctx, [("tiling", native.FD_STAGE_TILING),
                                                 ("topk", native.FD_STAGE_TOPK),
                                                 ("fuse", native.FD_STAGE_FUSE)])
        ff = torch.isfinite(fc) & fin
        fpmvo = {"points_per_s": sc.n_points / (el_f / args.steps),
                 "ms_per_step": el_f * 1e3 / args.steps, "stages_ms_per_launch": st_f,
                 "finite_frac": float(torch.isfinite(fc).float().mean()),
                 "mean_cost": float(fc[ff].mean()), "mean_cost_plain": float(costs[ff].mean()),
                 "err_vs_gt_deg": {"mean": float(_axial_deg(fd[ff], gt[ff]).mean()),
                                   "median": float(_axial_deg(fd[ff], gt[ff]).median())},
                 "mean_err_vs_plain_deg": float(_axial_deg(fd[ff], dirs[ff]).mean())}
        log(f"fpmvo (paper candidates): {fpmvo['points_per_s'] / 1e6:.1f} M points/s, "
            f"{json.dumps({k: round(v, 4) for k, v in st_f.items()})}, GT err median "
            f"{fpmvo['err_vs_gt_deg']['median']:.1f} deg (plain {float(err_gt.median()):.1f})")
    log(f"steps {args.steps}: {ms_step:.3f} ms/step, {value / 1e6:.1f} M points/s; "
        f"stages (ms/launch) {json.dumps({k: round(v, 4) for k, v in stages.items()})}; "
        f"finite costs {np.isfinite(c).mean():.4f}")
    out = {
        "metric": METRIC, "value": value, "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plain: 500k points, 20k strands, 64 views 1024^2 f16 maps, "
                               "10% outliers, P=5, 128 candidates + 8 refinement iterations",
                   "mode": "plain", "points": sc.n_points, "views": sc.n_views,
                   "depth_test": not args.no_depth,
                   "map": f"{sc.width}x{sc.height} f16", **kw},
        "roofline": {"bound": "alu", "kernel": "k_fuse", "achieved": achieved,
                     "peak": PEAK_FP32, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32,
                     "traffic": traffic_of("k_fuse, realistic 500k"),
                     "avg_launch_ms": stages["fuse"],
                     "flop_per_point": flop, "flop_per_sim_eval": FLOP_PER_SIM_EVAL},
        "stages_ms_per_launch": stages,
        "err_vs_gt_deg": {"mean": float(err_gt.mean()), "median": float(err_gt.median())},
        "fpmvo_paper_candidates": fpmvo,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, kw, args.cpu_seconds, depth=not args.no_depth)
        log(f"cpu baseline: {out['cpu_baseline']}")
    return out


def gabor_flop_per_pixel(n_orient, radius):
    """Algorithmic flop of the filter bank per pixel: one fma (2 flop) per
    tap and orientation; the argmax and the confidence are not counted."""
    return 2 * n_orient * (2 * radius + 1) ** 2


def run_gabor(args):
    import numpy as np
    import torch
    import oracle
    import scenegen
    from paper_2604_05794_amd import native

    name = "realistic"
    rec = scenegen.RECIPES[name]
    n_orient, radius = 32, 8
    t = time.perf_counter()
    frames, _, _, cams = scenegen.make_frames(name, args.seed)
    sc = scenegen.make_scene(name, args.seed)
    assert np.array_equal(cams, sc.cams)
    V, H, W = frames.shape
    log(f"generated {V} frames {W}x{H} and {sc.n_points} points in "
        f"{time.perf_counter() - t:.1f} s")
    dev = torch.device("cuda:0")
    fr = torch.from_numpy(frames).to(dev)
    th = torch.empty((V, H, W), dtype=torch.float16, device=dev)
    cf = torch.empty_like(th)
    ctx = native.Context(max_points=sc.n_points)
    stream = torch.cuda.current_stream()

    def step():
        native.orientation_maps(fr, n_orient=n_orient, radius=radius, theta=th, conf=cf,
                                out_dtype=torch.float16, stream=stream, ctx=ctx)

    el, stages = _timed(step, args, ctx, [("gabor", native.FD_STAGE_GABOR),
                                          ("gabor_norm", native.FD_STAGE_GABOR_NORM)])
    ms_step = el * 1e3 / args.steps
    px = V * H * W
    value = px / (el / args.steps)
    flop = gabor_flop_per_pixel(n_orient, radius)
    achieved = flop * px / (stages["gabor"] * 1e-3) / 1e12
    log(f"maps: {ms_step:.3f} ms/step, {value / 1e9:.2f} G pixels/s, "
        f"stages {json.dumps({k: round(v, 4) for k, v in stages.items()})}")
    # the direction search of the plain workload on the extracted maps
    kw = dict(patch=rec["patch"], n_candidates=rec["n_candidates"],
              refine_iters=rec["refine_iters"], top_k=5)
    pts = torch.from_numpy(sc.points).to(dev)
    cm = torch.from_numpy(sc.cams).to(dev)
    dm = torch.from_numpy(sc.depth.astype(np.float16)).to(dev)
    dirs = torch.empty((sc.n_points, 3), dtype=torch.float32, device=dev)
    costs = torch.empty((sc.n_points,), dtype=torch.float32, device=dev)

    def pipe():
        step()
        native.fuse_directions(pts, cm, th, cf, dirs=dirs, costs=costs, ctx=ctx, stream=stream,
                               depth_maps=dm, **kw)

    el_p, _ = _timed(pipe, args, ctx, [], profile=False)
    gt = torch.from_numpy(sc.gt).to(dev)
    fin = torch.isfinite(costs)
    err = _axial_deg(dirs[fin], gt[fin])
    pipeline = {"points_per_s": sc.n_points / (el_p / args.steps),
                "ms_per_step": el_p * 1e3 / args.steps,
                "finite_frac": float(fin.float().mean()),
                "err_vs_gt_deg": {"mean": float(err.mean()), "median": float(err.median())}}
    log(f"frames -> maps -> search: {json.dumps(pipeline)}")
    out = {
        "metric": "orientation-map pixels/s (Gabor bank, 32 orientations, radius 8)",
        "value": value, "unit": "pixels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"gabor: {V} grey frames {W}x{H} f32 -> f16 maps, "
                               f"{n_orient} orientations, radius {radius}",
                   "frames": V, "width": W, "height": H, "n_orient": n_orient,
                   "radius": radius},
        "roofline": {"bound": "mfma", "kernel": "k_gabor_mfma", "achieved": achieved,
                     "peak": PEAK_FP32_MFMA, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_MFMA,
                     "traffic": traffic_of("k_gabor_mfma, 64 frames 1024^2"),
                     "avg_launch_ms": stages["gabor"], "flop_per_pixel": flop},
        "stages_ms_per_launch": stages,
        "pipeline_frames_maps_search": pipeline,
    }
    if not args.no_cpu_baseline:
        bank = oracle.gabor_bank(n_orient=n_orient, radius=radius)
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
        threads = min(threads, os.cpu_count() or threads)
        done = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < args.cpu_seconds:
            oracle.gabor(frames[done % V], bank, n_threads=threads)
            done += 1
        el_c = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": done * H * W / el_c, "unit": "pixels/s",
                               "cores": threads, "kind": "oracle",
                               "sample": f"{done} whole frames of the same set, {el_c:.1f} s, "
                                         "binary64 oracle, OpenMP over pixels"}
        log(f"cpu baseline: {out['cpu_baseline']}")
    return out


def run_volume(args):
    import numpy as np
    import torch
    import oracle
    import scenegen
    from paper_2604_05794_amd import native

    n_pts, voxel = 2_000_000, 0.002
    t = time.perf_counter()
    pts, dirs, w, gt = scenegen.make_oriented_points("realistic", args.seed, n_pts)
    origin, h, dims = scenegen.head_grid(pts, voxel)
    nv = int(np.prod(dims.astype(np.int64)))
    log(f"generated {n_pts} oriented points, grid {dims.tolist()} ({nv} voxels) in "
        f"{time.perf_counter() - t:.1f} s")
    dev = torch.device("cuda:0")
    P = torch.from_numpy(pts).to(dev)
    D = torch.from_numpy(dirs).to(dev)
    W = torch.from_numpy(w).to(dev)
    shape = (int(dims[2]), int(dims[1]), int(dims[0]))
    occ = torch.empty(shape, dtype=torch.int32, device=dev)
    vd = torch.empty(shape + (3,), dtype=torch.float32, device=dev)
    vc = torch.empty(shape, dtype=torch.float32, device=dev)
    ctx = native.Context()
    stream = torch.cuda.current_stream()

    def step():
        native.fuse_volume(P, D, origin, h, dims, weights=W, occ=occ, dir_out=vd, coherence=vc,
                           stream=stream, ctx=ctx)

    stages_list = [("clear", native.FD_STAGE_VOLUME_CLEAR),
                   ("sort", native.FD_STAGE_VOLUME_SCATTER),
                   ("reduce", native.FD_STAGE_VOLUME_FINAL)]
    el, stages = _timed(step, args, ctx, stages_list)
    ms_step = el * 1e3 / args.steps
    value = n_pts / (el / args.steps)
    busy = int((occ > 0).sum())
    # algorithmic HBM bytes per launch (each array touched once): clear
    # writes the counts (4 B per voxel); sort reads the points (12 B), writes
    # voxel and rank (8 B), scans the counts into offsets (8 B read, 4 B
    # written per voxel) and places each point (voxel and rank 8 B, offset
    # 4 B, direction and weight 16 B read; 48 B of terms written); reduce
    # reads count and offset per voxel (8 B) and the terms of each point
    # (48 B) and writes orientation and coherence (16 B per voxel)
    alg = {"clear": 4 * nv, "sort": 96 * n_pts + 12 * nv, "reduce": 24 * nv + 48 * n_pts}
    gbs = {k: alg[k] / (stages[k] * 1e-3) / 1e9 for k in alg}
    dom = max(stages, key=lambda k: stages[k])
    kname = {"clear": "k_fill_u32 (counts)", "sort": "k_vol_key + scan + k_vol_place",
             "reduce": "k_vol_reduce"}[dom]
    log(f"volume: {ms_step:.3f} ms/step, {value / 1e6:.1f} M points/s, busy voxels {busy}, "
        f"stages {json.dumps({k: round(v, 4) for k, v in stages.items()})}, "
        f"GB/s {json.dumps({k: round(v, 1) for k, v in gbs.items()})}")
    # accuracy of the volume against the ground-truth tangents: the
    # orientation of each busy voxel vs the mean ground-truth line there
    gtv = oracle.volume(pts, gt, origin, h, dims)["dir"].reshape(-1, 3)
    got = vd.reshape(-1, 3).cpu().numpy().astype(np.float64)
    sel = np.any(gtv != 0, axis=1) & np.any(got != 0, axis=1)
    ang = np.degrees(np.arctan2(np.linalg.norm(np.cross(gtv[sel], got[sel]), axis=1),
                                np.abs(np.sum(gtv[sel] * got[sel], 1))))
    out = {
        "metric": "oriented points fused into the occupancy / orientation volume per second",
        "value": value, "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64 (int64 fixed-point sums)",
        "data": "synthetic",
        "config": {"workload": f"volume: {n_pts} oriented points of the realistic hairstyle, "
                               f"2 mm voxels, grid {dims.tolist()}",
                   "points": n_pts, "voxel_m": float(h), "dims": dims.tolist(),
                   "voxels": nv, "busy_voxels": busy},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": gbs[dom],
                     "peak": PEAK_HBM, "unit": "GB/s", "frac": gbs[dom] / PEAK_HBM,
                     "traffic": traffic_of(f"volume {dom}, realistic 2M points 2 mm"),
                     "avg_launch_ms": stages[dom], "algorithmic_bytes": alg[dom]},
        "stages_ms_per_launch": stages,
        "stages_GB_per_s": gbs,
        "orientation_err_vs_gt_deg": {"mean": float(ang.mean()), "median": float(np.median(ang))},
    }
    if not args.no_cpu_baseline:
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
        threads = min(threads, os.cpu_count() or threads)
        done = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < args.cpu_seconds:
            oracle.volume(pts, dirs, origin, h, dims, weights=w, n_threads=threads)
            done += 1
        el_c = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": done * n_pts / el_c, "unit": "points/s",
                               "cores": threads, "kind": "oracle",
                               "sample": f"{done} whole volumes of the same {n_pts} points, "
                                         f"{el_c:.1f} s, binary64 oracle (sums in one thread, "
                                         "eigenvectors with OpenMP)"}
        log(f"cpu baseline: {out['cpu_baseline']}")
    return out


def run_phg(args):
    import numpy as np
    import torch
    import oracle
    import scenegen
    from paper_2604_05794_amd import native

    n_pts, voxel, stride = 8_000_000, 0.003, 3
    grow_kw = dict(step=1e-3, max_steps=200, min_coherence=0.1,
                   max_bend_cos=math.cos(math.radians(45.0)), voxel_cap=8)
    link_kw = dict(max_dist=3e-3, min_cos=math.cos(math.radians(30.0)))
    t = time.perf_counter()
    pts, dirs, w, _ = scenegen.make_oriented_points("realistic", args.seed, n_pts)
    origin, h, dims = scenegen.head_grid(pts, voxel)
    roots, normals = scenegen.scalp_seeds("realistic", args.seed)
    lat = scenegen.lattice_seeds(origin, h, dims, stride)
    nv = int(np.prod(dims.astype(np.int64)))
    log(f"generated {n_pts} oriented points, grid {dims.tolist()}, {len(roots)} roots, "
        f"{len(lat)} segment seeds in {time.perf_counter() - t:.1f} s")
    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ctx = native.Context()
    stream = torch.cuda.current_stream()
    occ, vd, vc = native.fuse_volume(T(pts), T(dirs), origin, h, dims, weights=T(w), ctx=ctx,
                                     stream=stream)
    del pts, dirs, w
    R, Nr, L = T(roots), T(normals), T(lat)
    cr = torch.zeros(nv, dtype=torch.int32, device=dev)
    ng, ns = len(roots), len(lat)
    ar_g = torch.arange(ng, device=dev)
    ar_s = torch.arange(ns, device=dev)
    # room for every strand at its longest: all traces at full length
    S1 = grow_kw["max_steps"] + 1
    strands = torch.empty((ng * S1 + 2 * ns * S1, 3), dtype=torch.float32, device=dev)
    out = {}

    def step():
        cr.zero_()
        g = native.grow_strands(occ, vd, vc, origin, h, dims, R, Nr, crossings=cr, batch=4096,
                                stream=stream, ctx=ctx, **grow_kw)
        f = native.grow_strands(occ, vd, vc, origin, h, dims, L, None, crossings=cr,
                                batch=1 << 20, seed_mode=native.FD_SEED_AWAY, stream=stream,
                                ctx=ctx, **grow_kw)
        b = native.grow_strands(occ, vd, vc, origin, h, dims, L, None, crossings=cr,
                                batch=1 << 20, seed_mode=native.FD_SEED_TOWARDS, stream=stream,
                                ctx=ctx, **grow_kw)
        # the piece table: guide strands (no predecessor), then segments
        # (backward half reversed, then forward half)
        gn, fn, bn = g[1].long(), f[1].long(), b[1].long()
        S = torch.cat([R, b[0][ar_s, bn - 1]])
        SD = torch.cat([Nr, b[2]])
        E = torch.cat([g[0][ar_g, gn - 1], f[0][ar_s, fn - 1]])
        ED = torch.cat([g[2], f[2]])
        F = torch.cat([(gn > 1).to(torch.uint8), ((fn > 1) & (bn > 1)).to(torch.uint8) * 3])
        succ = native.link_segments(S, SD, E, ED, F, stream=stream, ctx=ctx, **link_kw)
        off, _, pieces = native.assemble_strands(g, f, b, succ, out=strands, stream=stream,
                                                 ctx=ctx)
        out.update(g=g, f=f, b=b, succ=succ, F=F, off=off, pieces=pieces)

    stages_list = [("grow", native.FD_STAGE_GROW), ("crossings", native.FD_STAGE_GROW_CROSS),
                   ("link", native.FD_STAGE_LINK)]
    el, stages = _timed(step, args, ctx, stages_list)
    n_launch = {"grow": math.ceil(ng / 4096) + 2, "crossings": math.ceil(ng / 4096) + 2,
                "link": 1}
    per_step = {k: stages[k] * n_launch[k] for k in stages}
    ms_step = el * 1e3 / args.steps
    g, f, b, succ, F = out["g"], out["f"], out["b"], out["succ"], out["F"]
    gsteps = int((g[1] - 1).sum())
    ssteps = int((f[1] - 1).sum() + (b[1] - 1).sum())
    links = int((succ >= 0).sum())
    off, pieces = out["off"], out["pieces"]
    slen = (off[1:] - off[:-1]).float() * grow_kw["step"] * 1e3 - grow_kw["step"] * 1e3
    # algorithmic bytes of the growing kernel per step: the voxel's count,
    # coherence, crossing count and orientation (24 B) and the new vertex
    # (12 B); per strand the seed, its direction and the outputs (40 B)
    alg_grow = 36 * (gsteps + ssteps) + 40 * (ng + 2 * ns)
    grow_ms = per_step["grow"]
    achieved = alg_grow / (grow_ms * 1e-3) / 1e9
    value = ng / (el / args.steps)
    guide_len = (g[1] - 1).float() * grow_kw["step"] * 1e3
    log(f"phg: {ms_step:.3f} ms/step; per step (ms) {json.dumps({k: round(v, 4) for k, v in per_step.items()})}; "
        f"guide steps {gsteps}, segment steps {ssteps}, valid segments "
        f"{int((F[ng:] == 3).sum())}, links {links}")
    res = {
        "metric": "guide strands grown and linked per second (parallel hair growing)",
        "value": value, "unit": "strands/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"phg: {ng} scalp roots + {ns} interior seeds traced both ways "
                               f"through the 3 mm volume of {n_pts} oriented points, Eq. 13 "
                               "linking of all pieces",
                   "roots": ng, "segment_seeds": ns, "grid": dims.tolist(), "voxel_m": float(h),
                   **grow_kw, **link_kw, "batch": 4096},
        "roofline": {"bound": "hbm", "kernel": "k_grow", "achieved": achieved,
                     "peak": PEAK_HBM, "unit": "GB/s", "frac": achieved / PEAK_HBM,
                     "traffic": traffic_of("k_grow, phg workload"),
                     "avg_launch_ms": stages["grow"], "algorithmic_bytes_per_step": alg_grow,
                     "note": "dependent voxel lookups: latency-bound, not bandwidth-bound"},
        "stages_ms_per_launch": stages,
        "stages_ms_per_step": per_step,
        "result": {"strand_mean_length_mm": float(slen.mean()),
                   "strand_median_length_mm": float(slen.median()),
                   "strands_with_segments": int((pieces > 1).sum()),
                   "strand_vertices": int(off[-1]),
                   "guide_mean_length_mm": float(guide_len.mean()),
                   "guide_median_length_mm": float(guide_len.median()),
                   "guide_steps": gsteps, "segment_steps": ssteps,
                   "valid_segments": int((F[ng:] == 3).sum()), "links": links},
    }
    if not args.no_cpu_baseline:
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
        threads = min(threads, os.cpu_count() or threads)
        host = dict(occ=occ.cpu().numpy().view(np.uint32), dir=vd.cpu().numpy(),
                    coherence=vc.cpu().numpy())
        grid = (origin, h, dims)
        t0 = time.perf_counter()
        go = oracle.grow(host, grid, roots, normals, batch=4096, **grow_kw)
        fo = oracle.grow(host, grid, lat, None, crossings=go["crossings"], batch=1 << 20,
                         seed_mode=1, **grow_kw)
        bo = oracle.grow(host, grid, lat, None, crossings=fo["crossings"], batch=1 << 20,
                         seed_mode=2, **grow_kw)
        t_grow = time.perf_counter() - t0
        # linking: the pieces of a bounded sample of roots and segments (the
        # brute-force pair test is quadratic)
        gn, fn, bn = go["n_verts"], fo["n_verts"], bo["n_verts"]
        k = min(ns, 12000)
        S = np.concatenate([roots, bo["verts"][np.arange(k), bn[:k] - 1]])
        SD = np.concatenate([normals, bo["last_dir"][:k]])
        E = np.concatenate([go["verts"][np.arange(ng), gn - 1], fo["verts"][np.arange(k), fn[:k] - 1]])
        ED = np.concatenate([go["last_dir"], fo["last_dir"][:k]])
        Fo = np.concatenate([np.where(gn > 1, 1, 0), np.where((fn[:k] > 1) & (bn[:k] > 1), 3, 0)]).astype(np.uint8)
        t1 = time.perf_counter()
        oracle.link(S, SD, E, ED, Fo, link_kw["max_dist"], link_kw["min_cos"], n_threads=threads)
        t_link = time.perf_counter() - t1
        # scale the link time to all pieces by the quadratic pair count
        n_all = ng + ns
        t_link_all = t_link * (n_all / len(S)) ** 2
        res["cpu_baseline"] = {
            "value": ng / (t_grow + t_link_all), "unit": "strands/s", "cores": threads,
            "kind": "oracle",
            "sample": f"oracle growing of all {ng} roots and {ns} segment seeds both ways "
                      f"({t_grow:.2f} s, one thread) and its brute-force linking of "
                      f"{len(S)} of the {n_all} pieces ({t_link:.2f} s on {threads} threads), "
                      f"scaled by the pair count to {t_link_all:.1f} s for all pieces"}
        log(f"cpu baseline: {res['cpu_baseline']}")
    return res


PEAK_BF16_MFMA = 2500.0       # TFLOP/s, dense


def run_train(args):
    import numpy as np
    import torch
    import scenegen
    from paper_2604_05794_amd import native

    name = "realistic"
    rec = scenegen.RECIPES[name]
    sc = scenegen.make_scene(name, args.seed)
    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    pts, cams, th, cf, dm = T(sc.points), T(sc.cams), T(sc.theta), T(sc.conf), T(sc.depth)
    # the training pairs: proposal features and the plain search's directions
    feats = native.features(pts, cams, th, cf, head_centre=tuple(sc.head_centre), depth_maps=dm)
    dirs, costs = native.fuse_directions(pts, cams, th, cf, depth_maps=dm, patch=rec["patch"],
                                         n_candidates=rec["n_candidates"],
                                         refine_iters=rec["refine_iters"], top_k=5)
    ok = torch.isfinite(costs)
    feats, dirs = feats[ok].contiguous(), dirs[ok].contiguous()
    B = 4096
    nb = feats.shape[0] // B
    net = native.MLP(seed=args.seed)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    k = [0]

    def step():
        i = k[0] % nb
        k[0] += 1
        net.train_step(feats[i * B:(i + 1) * B], dirs[i * B:(i + 1) * B], lr=1e-3, loss=loss,
                       stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    l0 = float(loss)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    step_ms = ev0.elapsed_time(ev1) / args.steps
    # flop per sample: forward 2 x 160,512 MAC; weight gradients the same;
    # input gradients of layers 2-4 (layer 1's input needs none)
    mac = 112 * 256 + 256 * 256 + 256 * 256 + 256 * 3
    flop = 2 * mac * 3 - 2 * 112 * 256
    achieved = flop * B / (step_ms * 1e-3) / 1e12
    value = B * args.steps / el
    log(f"train: {step_ms:.3f} ms/step (batch {B}), {value / 1e6:.2f} M samples/s, "
        f"{achieved:.1f} TFLOP/s, loss {l0:.4f} -> {float(loss):.4f}")
    return {
        "metric": "proposal-network training samples per second (Adam, batch 4096)",
        "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": el * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16 (f32 master, accumulation)",
        "data": "synthetic",
        "config": {"workload": "train: 112-256-256-256-3 GELU network, batch 4096, features and "
                               "plain-search targets of the realistic scene",
                   "batch": B, "pairs": int(feats.shape[0])},
        "roofline": {"bound": "mfma", "kernel": "train step (k_gemm_bf16 GEMMs, loss, Adam)",
                     "achieved": achieved, "peak": PEAK_BF16_MFMA, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_BF16_MFMA, "traffic": None,
                     "avg_step_ms": step_ms, "flop_per_sample": flop},
        "loss": {"after_warmup": l0, "final": float(loss)},
    }


def run_pipeline(args):
    import numpy as np
    import torch
    import scenegen
    from paper_2604_05794_amd import native

    name = "realistic"
    rec = scenegen.RECIPES[name]
    t = time.perf_counter()
    frames, _, _, cams = scenegen.make_frames(name, args.seed)
    sc = scenegen.make_scene(name, args.seed)
    assert np.array_equal(cams, sc.cams)
    pin, din, win, _ = scenegen.make_oriented_points(name, args.seed + 1, 1_500_000)
    roots, normals = scenegen.scalp_seeds(name, args.seed)
    origin, h, dims = scenegen.head_grid(np.concatenate([sc.points, pin]), 0.003)
    lat = scenegen.lattice_seeds(origin, h, dims, 3)
    log(f"generated frames, {sc.n_points} outer + {len(pin)} inner points, grid "
        f"{dims.tolist()} in {time.perf_counter() - t:.1f} s")
    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    fr, pts, cm, dm = T(frames), T(sc.points), T(sc.cams), T(sc.depth)
    Pin, Din, Win = T(pin), T(din), T(win)
    R, Nr, L = T(roots), T(normals), T(lat)
    V, H, W = frames.shape
    n_out, ng, ns = sc.n_points, len(roots), len(lat)
    nv = int(np.prod(dims.astype(np.int64)))
    th = torch.empty((V, H, W), dtype=torch.float16, device=dev)
    cf = torch.empty_like(th)
    dirs = torch.empty((n_out, 3), dtype=torch.float32, device=dev)
    costs = torch.empty((n_out,), dtype=torch.float32, device=dev)
    allp = torch.cat([pts, Pin])
    alld = torch.empty((n_out + len(pin), 3), dtype=torch.float32, device=dev)
    allw = torch.cat([torch.ones(n_out, dtype=torch.float32, device=dev), Win])
    shape = (int(dims[2]), int(dims[1]), int(dims[0]))
    occ = torch.empty(shape, dtype=torch.int32, device=dev)
    vd = torch.empty(shape + (3,), dtype=torch.float32, device=dev)
    vc = torch.empty(shape, dtype=torch.float32, device=dev)
    cr = torch.zeros(nv, dtype=torch.int32, device=dev)
    gkw = dict(step=1e-3, max_steps=200, min_coherence=0.1,
               max_bend_cos=math.cos(math.radians(45.0)), voxel_cap=8)
    S1 = gkw["max_steps"] + 1
    strands = torch.empty((ng * S1 + 2 * ns * S1, 3), dtype=torch.float32, device=dev)
    ar_g = torch.arange(ng, device=dev)
    ar_s = torch.arange(ns, device=dev)
    ctx = native.Context(max_points=n_out)
    stream = torch.cuda.current_stream()
    kw = dict(patch=rec["patch"], n_candidates=rec["n_candidates"],
              refine_iters=rec["refine_iters"], top_k=5)
    res = {}

    def step():
        native.orientation_maps(fr, theta=th, conf=cf, out_dtype=torch.float16, stream=stream,
                                ctx=ctx)
        native.fuse_directions(pts, cm, th, cf, dirs=dirs, costs=costs, ctx=ctx, stream=stream,
                               depth_maps=dm, **kw)
        alld[:n_out].copy_(dirs)
        alld[n_out:].copy_(Din)
        native.fuse_volume(allp, alld, origin, h, dims, weights=allw, occ=occ, dir_out=vd,
                           coherence=vc, stream=stream, ctx=ctx)
        cr.zero_()
        g = native.grow_strands(occ, vd, vc, origin, h, dims, R, Nr, crossings=cr, batch=4096,
                                stream=stream, ctx=ctx, **gkw)
        f = native.grow_strands(occ, vd, vc, origin, h, dims, L, None, crossings=cr,
                                batch=1 << 20, seed_mode=native.FD_SEED_AWAY, stream=stream,
                                ctx=ctx, **gkw)
        b = native.grow_strands(occ, vd, vc, origin, h, dims, L, None, crossings=cr,
                                batch=1 << 20, seed_mode=native.FD_SEED_TOWARDS, stream=stream,
                                ctx=ctx, **gkw)
        gn, fn, bn = g[1].long(), f[1].long(), b[1].long()
        S = torch.cat([R, b[0][ar_s, bn - 1]])
        SD = torch.cat([Nr, b[2]])
        E = torch.cat([g[0][ar_g, gn - 1], f[0][ar_s, fn - 1]])
        ED = torch.cat([g[2], f[2]])
        F = torch.cat([(gn > 1).to(torch.uint8), ((fn > 1) & (bn > 1)).to(torch.uint8) * 3])
        succ = native.link_segments(S, SD, E, ED, F, 3e-3, math.cos(math.radians(30.0)),
                                    stream=stream, ctx=ctx)
        off, _, pieces = native.assemble_strands(g, f, b, succ, out=strands, stream=stream,
                                                 ctx=ctx)
        res.update(off=off, pieces=pieces)

    stages_list = [("gabor", native.FD_STAGE_GABOR), ("gabor_norm", native.FD_STAGE_GABOR_NORM),
                   ("tiling", native.FD_STAGE_TILING), ("topk", native.FD_STAGE_TOPK),
                   ("fuse", native.FD_STAGE_FUSE), ("volume_clear", native.FD_STAGE_VOLUME_CLEAR),
                   ("volume_sort", native.FD_STAGE_VOLUME_SCATTER),
                   ("volume_reduce", native.FD_STAGE_VOLUME_FINAL),
                   ("grow", native.FD_STAGE_GROW), ("crossings", native.FD_STAGE_GROW_CROSS),
                   ("link", native.FD_STAGE_LINK)]
    el, stages = _timed(step, args, ctx, stages_list)
    ms_step = el * 1e3 / args.steps
    n_launch = {"grow": math.ceil(ng / 4096) + 2, "crossings": math.ceil(ng / 4096) + 2}
    per_step = {k: v * n_launch.get(k, 1) for k, v in stages.items()}
    flop = gabor_flop_per_pixel(32, 8)
    px = V * H * W
    achieved = flop * px / (stages["gabor"] * 1e-3) / 1e12
    off, pieces = res["off"], res["pieces"]
    slen = (off[1:] - off[:-1]).float() - 1.0
    log(f"pipeline: {ms_step:.3f} ms per reconstruction; per step (ms) "
        f"{json.dumps({k: round(v, 4) for k, v in per_step.items()})}")
    return {
        "metric": "hair reconstructions per second on one GPU (frames -> maps -> directions -> "
                  "volume -> strands)",
        "value": 1e3 / ms_step, "unit": "reconstructions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"pipeline: {V} frames {W}x{H} -> maps -> {n_out} outer points "
                               f"searched -> volume of {n_out + len(pin)} points at 3 mm -> "
                               f"{ng} roots + {ns} segment seeds -> linked strands",
                   "frames": V, "outer_points": n_out, "inner_points": len(pin),
                   "grid": dims.tolist(), "roots": ng, "segment_seeds": ns},
        "roofline": {"bound": "mfma", "kernel": "k_gabor_mfma (the longest stage)",
                     "achieved": achieved, "peak": PEAK_FP32_MFMA, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_MFMA,
                     "traffic": traffic_of("k_gabor_mfma, 64 frames 1024^2"),
                     "avg_launch_ms": stages["gabor"]},
        "stages_ms_per_step": per_step,
        "result": {"strand_vertices": int(off[-1]), "strands_with_segments":
                   int((pieces > 1).sum()), "strand_mean_steps": float(slen.mean())},
    }


def run_gains(args):
    """What the network gains over the method without it, and what the
    threshold trades.  On the realistic scene and one tight-curl head:
    the learned form with the network proposal against the learned form with
    a proposal from a small Fibonacci lattice (N' directions, no refinement:
    the plain search with n_candidates = N', refine_iters = 0), both refined
    by the same 2 iterations from the same calibrated step and held to the
    same threshold tau (equal sim-eval budget after the proposal); N' runs
    over a range and the one whose proposal takes the network's measured
    time (features + forward) is marked.  Then a sweep of tau for the
    network form.  Each row: points/s of the whole learned call (proposal
    included), fallback fraction, mean and 95th-percentile angle to the plain
    result."""
    import numpy as np
    import torch
    import scenegen
    from paper_2604_05794_amd import native

    dev = torch.device("cuda:0")
    net = native.MLP(path=args.mlp)
    step0, tau0 = net.calibration()
    stream = torch.cuda.current_stream()
    out = {"workload": "network proposal vs Fibonacci proposal at equal refinement budget; "
                       "threshold sweep", "learned_step0": step0, "tau_calibrated": tau0,
           "scenes": {}}

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps

    for name in ("realistic", "curls"):
        rec = scenegen.RECIPES[name]
        kw = dict(patch=rec["patch"], n_candidates=rec["n_candidates"],
                  refine_iters=rec["refine_iters"], top_k=5)
        sc = scenegen.make_scene(name, args.seed)
        n = sc.n_points
        pts, cams = torch.from_numpy(sc.points).to(dev), torch.from_numpy(sc.cams).to(dev)
        th, cf = torch.from_numpy(sc.theta).to(dev), torch.from_numpy(sc.conf).to(dev)
        kw["depth_maps"] = torch.from_numpy(sc.depth).to(dev)
        ctx = native.Context(max_points=n, max_views=sc.n_views)
        dp, cp = (torch.empty((n, 3), device=dev), torch.empty((n,), device=dev))
        dl, cl = torch.empty_like(dp), torch.empty_like(cp)
        dq, cq = torch.empty_like(dp), torch.empty_like(cp)

        def plain():
            native.fuse_directions(pts, cams, th, cf, dirs=dp, costs=cp, ctx=ctx, stream=stream,
                                   **kw)
        t_plain = timed(plain)
        fin = torch.isfinite(cp)

        def row(t, d):
            a = _axial_deg(d[fin], dp[fin])
            return {"points_per_s": n / t, "ms": t * 1e3, "fallback": ctx.fallback_count() / n,
                    "mean_err_vs_plain_deg": float(a.mean()),
                    "p95_err_vs_plain_deg": float(torch.quantile(a, 0.95))}

        def learned_net(tau):
            def fn():
                native.fuse_directions(pts, cams, th, cf, dirs=dl, costs=cl, ctx=ctx,
                                       stream=stream, mode=native.FD_MODE_LEARNED, mlp=net,
                                       learned_iters=2, learned_step0=step0, fallback_cost=tau,
                                       head_centre=sc.head_centre, **kw)
            return fn
        t_net = timed(learned_net(tau0))
        res = {"plain": {"points_per_s": n / t_plain, "ms": t_plain * 1e3},
               "network": row(t_net, dl)}
        st = _stage_pass(learned_net(tau0), ctx, [("features", native.FD_STAGE_FEATURES),
                                                 ("mlp", native.FD_STAGE_MLP)])
        t_prop_net = (st.get("features", 0.0) + st.get("mlp", 0.0)) * 1e-3
        res["network"]["proposal_ms"] = t_prop_net * 1e3
        fib = {}
        for nprime in (4, 8, 12, 16, 24, 32, 48, 64):
            pkw = dict(kw, n_candidates=nprime, refine_iters=0)

            def prop():
                native.fuse_directions(pts, cams, th, cf, dirs=dq, costs=cq, ctx=ctx,
                                       stream=stream, **pkw)

            def fn():
                prop()
                native.fuse_directions(pts, cams, th, cf, dirs=dl, costs=cl, ctx=ctx,
                                       stream=stream, mode=native.FD_MODE_LEARNED,
                                       proposal=native.FD_PROPOSAL_GIVEN, proposal_dirs=dq,
                                       learned_iters=2, learned_step0=step0, fallback_cost=tau0,
                                       **kw)
            t_prop = timed(prop)
            t_all = timed(fn)
            r = row(t_all, dl)
            r["proposal_ms"] = t_prop * 1e3
            fib[nprime] = r
        res["fibonacci"] = fib
        match = min(fib, key=lambda k: abs(fib[k]["proposal_ms"] - t_prop_net * 1e3))
        res["fibonacci_matched_n"] = match
        sweep = {}
        for tau in sorted({0.5 * tau0, tau0, 1.5 * tau0, 2 * tau0, 3 * tau0, 0.1, 0.2, 0.3}):
            t = timed(learned_net(tau))
            sweep[f"{tau:.4f}"] = row(t, dl)
        t = timed(learned_net(float("inf")))
        sweep["inf"] = row(t, dl)
        res["tau_sweep"] = sweep
        out["scenes"][name] = res
        log(f"{name}: plain {n / t_plain / 1e6:.1f} M points/s; network "
            f"{json.dumps({k: round(v, 4) for k, v in res['network'].items()})}; fibonacci "
            f"N'={match} {json.dumps({k: round(v, 4) for k, v in fib[match].items()})}")
    return out


def l2_probe(sizes=(1 << 20, 2 << 20, 3 << 20), blocks=2048, target_bytes=16 << 30):
    """Aggregate read bandwidth of buffers that fit one XCD's L2 (4 MiB):
    every workgroup reads the whole buffer (fd_probe_read), so every XCD
    serves it from its own L2.  GB/s per size, best of 5 launches."""
    import torch
    from paper_2604_05794_amd import native
    out = {}
    sink = torch.empty(blocks * 256, dtype=torch.int32, device="cuda:0")
    for nb in sizes:
        buf = torch.ones(nb // 4, dtype=torch.int32, device="cuda:0")
        reps = max(1, int(target_bytes // (nb * blocks)))
        native.probe_read(buf, reps, blocks, sink)  # warm the caches
        best = 0.0
        for _ in range(5):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            native.probe_read(buf, reps, blocks, sink)
            b.record()
            b.synchronize()
            best = max(best, nb * reps * blocks / (a.elapsed_time(b) * 1e-3) / 1e9)
        out[f"{nb >> 20}MiB"] = best
    return out


def run_l2(args):
    """Read-bandwidth ceilings: L2-resident buffers (every XCD reads its own
    copy from L2) and, for scale, buffers in the last-level MALL."""
    res = l2_probe()
    mall = l2_probe(sizes=(64 << 20,), blocks=256)
    log(f"L2 probe {json.dumps({k: round(v) for k, v in res.items()})} GB/s; MALL {mall}")
    return {"workload": "read bandwidth probe", "l2_GB_per_s": res, "mall_GB_per_s": mall,
            "l2_peak_measured_GB_per_s": max(res.values())}


def run_copy(args):
    """Counter calibration: a plain device-to-device copy of 512 MiB, so the
    FETCH_SIZE / WRITE_SIZE counters can be read against known bytes."""
    import torch
    n = 512 << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return {"workload": "copy calibration", "bytes_read_per_copy": n, "bytes_written_per_copy": n,
            "copies": args.steps, "GB_per_s": 2 * n * args.steps / el / 1e9}


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workload", default="metric",
                    choices=["metric", "plain", "learned", "gabor", "volume", "phg", "train",
                             "pipeline", "copy", "l2", "gains", "batched"])
    ap.add_argument("--heads", type=int, default=8)
    ap.add_argument("--mlp", default=os.path.join(ROOT, "paper_2604_05794_amd", "weights",
                                                  "proposal_mlp.fdmlp"))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-depth", action="store_true",
                    help="run without the depth visibility test")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE "
              f"{world}); the fusion shards by scene or by point range with no exchange, and "
              "this build runs the one-GPU share.", file=sys.stderr)
        sys.exit(2)
    run = {"metric": run_metric, "plain": run_plain, "learned": run_learned,
           "gabor": run_gabor, "volume": run_volume, "phg": run_phg, "train": run_train,
           "pipeline": run_pipeline,
           "copy": run_copy, "l2": run_l2, "gains": run_gains,
           "batched": run_batched}[args.workload]
    out = run(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
