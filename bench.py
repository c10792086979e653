"""Benchmark: forward+backward pixel-primitive pairs per second of the
splattable-neural-primitive rasterizer on one MI355X.

A step is one whole pass of the path: preprocess (bounds, keys, records,
colour MLP), tile binning, radix sort, tile ranges, forward rasterizer, L1
loss, backward rasterizer, colour-MLP and preprocess adjoints.  The default
workload is 16 cameras of mixed resolution (4 x 640x480, 8 x 1280x720,
4 x 1920x1080) looking at 200k primitives (density MLP N=16, colour MLP
width 32 depth 2), run as ONE HIP graph with persistent rasterizer launches.

Printed (one JSON line): the metric value = forward hit pairs per step /
seconds per step; ms/step of the batched graph and of per-view plain
launches (same kernels, one camera at a time, no graph, no persistence);
the roofline of the dominant kernel (the rasterizer backward, measured live
with HIP events around its launches); and the FP64 oracle timed on a
bounded crop of the same workload on the host's cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_SLOTS = 256 * 128 * 2.4e9   # FP32 VALU lane-op issue slots/s (= 157.3 TFLOP/s / 2)
TRANS_WEIGHT = 4.0               # issue slots per transcendental (quarter rate)


def ops_per_pair(N, ray_colour_width=0):
    """Algorithmic work of the rasterizer per pair, in VALU lane-ops and
    transcendentals, counted from the formulation (ray frame and
    discriminant, chord, per hidden unit the phase, half-width, cos, sin,
    reciprocal and sinc, then alpha and blending): forward per hit pair;
    backward per hit pair plus per live pair (pairs with a positive,
    unclamped integral, which carry gradient)."""
    fwd_v, fwd_t = 50 + 11 * N, 3 * N + 3
    bwd_hit_v, bwd_hit_t = fwd_v + 25, fwd_t
    # with the forward's pair integrals at hand, a hit pair in the backward
    # needs the chord only (ray frame, discriminant, sqrt, 1/A: 26 ops + 2),
    # alpha (exp2) and the blending and d loss / d integral (40 ops + 1/H)
    bwd_hit_cached_v, bwd_hit_cached_t = 66, 4
    bwd_live_v, bwd_live_t = 32 * N + 60, 6 * N + 1
    if ray_colour_width:
        # the per-ray colour network (one hidden layer of W units) per pair:
        # entry point and direction (6 ops + 1/L), first layer (6 FMA + ReLU
        # per unit), output layer (3 W FMA), sigmoid (2 ops + exp2 + rcp per
        # channel), c_dc (3); in the backward's pixel phase again, and per
        # listed pair the recomputation plus its adjoint: sigmoid derivative
        # (4 per channel), output weights (3 W), hidden gradient (3 FMA +
        # select per unit), first-layer weights (6 W) and the entry point
        # and direction gradients (6 W FMA), 9 more in the geometry chain
        W = ray_colour_width
        col = (10 * W + 15, 7)
        fwd_v, fwd_t = fwd_v + col[0], fwd_t + col[1]
        bwd_hit_v, bwd_hit_t = bwd_hit_v + col[0], bwd_hit_t + col[1]
        bwd_hit_cached_v, bwd_hit_cached_t = bwd_hit_cached_v + col[0], bwd_hit_cached_t + col[1]
        bwd_live_v, bwd_live_t = bwd_live_v + col[0] + 21 + 19 * W, bwd_live_t + col[1]
    return dict(fwd=(fwd_v, fwd_t), bwd_hit=(bwd_hit_v, bwd_hit_t), bwd_hit_cached=(bwd_hit_cached_v, bwd_hit_cached_t),
                bwd_live=(bwd_live_v, bwd_live_t))


def slots(vt):
    return vt[0] + TRANS_WEIGHT * vt[1]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="C4", choices=["C3", "C4", "C5", "R", "L", "D", "A"],
                    help="C3/C4/C5: fwd+bwd step; R: the C4 step with the per-ray relighting colour; "
                         "L: the C4 step with the relighting colour per (primitive, view); "
                         "D: the C4 step with the dynamic-scene density and SH colour; "
                         "A: forward-only frames/s of the 100k-primitive throughput workload")
    ap.add_argument("--tile", default=None, help="tile_w,tile_h,px_per_lane[,bwd_batch] (default: tuned)")
    ap.add_argument("--fwd-cache", type=int, default=None, choices=[0, 1],
                    help="1: the forward keeps every pair's integral for the backward; 0: the backward "
                         "re-evaluates (default: 1 for C3/C4, 0 for C5, whose step recomputes per-tile state)")
    ap.add_argument("--bin-order", type=int, default=0, choices=[0, 1, 2],
                    help="1 depth sort of the pairs then tile-bit instance sort, 2 full-key sort, 0 by size")
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-check", action="store_true")
    ap.add_argument("--oracle-views", type=int, default=16,
                    help="views whose sampled tile is checked against the oracle (one tile per view)")
    ap.add_argument("--oracle-tiles-per-view", type=int, default=1,
                    help="tiles of each checked view compared with the oracle")
    ap.add_argument("--oracle-grad-primitives", type=int, default=0,
                    help="primitives whose gradients from one step are checked against the oracle (0: none)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--eager-only", action="store_true",
                    help="profiling aid: only run --steps eager steps (no graph, no per-view, no CPU leg) and print timings")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU only: the path would shard over the "
                                   "views, with one gradient reduction per step; run with --gpus 1"}))
        sys.exit(2)

    import torch
    import synthetic as S

    if a.workload == "A":
        torch.cuda.set_device(0)
        return forward_fps(a)
    cfg0, scene, cams, targets = S.make_workload(a.workload)
    fwd_cache = a.fwd_cache if a.fwd_cache is not None else (0 if a.workload == "C5" else 1)

    # ---- the oracle on the host's cores, before the GPU is touched (the
    # worker processes are forked from a process without a GPU context) -----------
    grad_ref = None
    if a.oracle_grad_primitives > 0:
        grad_ref = oracle_grad_reference(scene, cams, targets, a.oracle_grad_primitives)
        log(f"[bench] oracle gradients of {len(grad_ref['primitives'])} primitives over "
            f"{len(grad_ref['windows'])} windows in {grad_ref['seconds']} s")
    cpu = None
    if not a.no_cpu_baseline and not a.eager_only:
        cpu = cpu_baseline(scene, cams, targets, a.cpu_seconds, a.workload)
        log(f"[bench] cpu oracle: {cpu}")

    import paper_2510_08491_amd as snp
    from paper_2510_08491_amd import tuning
    import paper_2510_08491_amd.render as rmod

    torch.cuda.set_device(0)
    N = scene["N"]
    if a.tile:
        tile = tuple(int(x) for x in a.tile.split(","))
    else:
        tile = tuning.lookup(N, scene["color_mode"], cams, fwd_cache) or (16, 16, 1)
    if len(tile) == 3:
        tile = tile + (0,)
    cfg = snp.RenderConfig(n_hidden=N, omega0=scene["omega0"], color_mode=scene["color_mode"], bin_order=a.bin_order,
                           cmlp_width=scene["cmlp_width"], cmlp_depth=scene["cmlp_depth"], tile_w=tile[0],
                           tile_h=tile[1], px_per_lane=tile[2], bwd_batch=tile[3], persistent=1, fwd_cache=fwd_cache,
                           time=float(scene.get("time", 0.0)))
    log(f"[bench] workload {a.workload}: P={scene['P']} V={len(cams)} N={N} tile={tile} fwd_cache={fwd_cache}")
    params = snp.params_to_device(scene)
    tg = torch.from_numpy(np.concatenate([t.ravel() for t in targets])).cuda()
    n_norm = float(tg.numel())

    # size the workspace from one binning pass, then count pairs (untimed)
    rast = snp.Rasterizer(cfg, scene["P"], cams)
    inst = rast.prepare(params)
    rast._alloc(int(inst * 1.1) + 4096)
    rast.prepare(params)
    images, final_T = rast.new_images()
    rast.forward(params, images, final_T, count_pairs=True)
    cnt = rast.counters()
    hit_pairs, live_pairs = cnt["hit_pairs"], cnt["live_pairs"]
    tile_pairs = rast.tile_pairs().cpu().numpy().astype(np.int64)
    log(f"[bench] instances {inst}, hit pairs {hit_pairs}, live pairs {live_pairs}, "
        f"pair cache {rast.fwd_cache} ({rast.layout.ahat_cache_bytes / 2 ** 30:.1f} GiB, "
        f"{rast.cached_instances} of {inst} instances)")
    if a.eager_only:
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        dL = torch.empty_like(images)
        grads = snp.zeros_like_params(params)
        for s in range(a.steps):
            t0 = time.perf_counter()
            rast.step(params, images, final_T, tg, n_norm, loss, dL, grads)
            torch.cuda.synchronize()
            log(f"[bench] eager step {s}: {1e3 * (time.perf_counter() - t0):.1f} ms")
        rast.read_status()
        return

    # ---- batched: one graph per step -------------------------------------------------
    step = snp.GraphStep(rast, params, tg, n_norm)
    for _ in range(a.warmup):
        step.launch()
    torch.cuda.synchronize()
    log("[bench] warmup done")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for _ in range(a.steps):
        step.launch()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = e0.elapsed_time(e1) / a.steps
    # the replays' device flags: instance overflow, phase range (raises on either)
    step.check()
    status_ok = True
    log(f"[bench] batched graph: {ms_step:.3f} ms/step (wall {1e3 * wall / a.steps:.3f}), status ok")
    img_batched = step.images.clone()

    # ---- rasterizer kernels timed live (eager step, HIP events on the launch stream) --
    fwd_ms, bwd_ms = eager_kernel_ms(snp, rmod, torch, rast, params, images, final_T, tg, n_norm, a.steps)
    log(f"[bench] raster kernels: forward {fwd_ms:.3f} ms, backward {bwd_ms:.3f} ms")
    pair_cache = rast.fwd_cache
    cache_gb = rast.layout.ahat_cache_bytes / 2 ** 30
    cached_frac = rast.cached_instances / max(inst, 1) if pair_cache else 0.0
    del step, rast, images, final_T
    torch.cuda.empty_cache()

    # ---- the oracle on sampled tiles of the batched images (untimed) -----------------
    check = None
    if not a.no_oracle_check:
        check = oracle_check(scene, cams, cfg, img_batched, tile_pairs, a.oracle_views, a.oracle_tiles_per_view)
        log(f"[bench] oracle check: {check}")

    # ---- the same step re-evaluating every pair in the backward (no pair cache) --------
    recompute = None
    if pair_cache:
        cfg_rc = snp.RenderConfig(**{**cfg.__dict__, "fwd_cache": 0})
        r0 = snp.Rasterizer(cfg_rc, scene["P"], cams)
        r0._alloc(int(r0.prepare(params) * 1.1) + 4096)
        im0, T0 = r0.new_images()
        f_rc, b_rc = eager_kernel_ms(snp, rmod, torch, r0, params, im0, T0, tg, n_norm, a.steps)
        same = bool(torch.equal(im0, img_batched))
        del r0, im0, T0
        torch.cuda.empty_cache()
        recompute = {"fwd_ms": round(f_rc, 4), "bwd_ms": round(b_rc, 4), "images_identical": same}
        log(f"[bench] without the pair cache: forward {f_rc:.3f} ms, backward {b_rc:.3f} ms, images identical {same}")

    grad_check = None
    if grad_ref is not None:
        grad_check = oracle_grad_check(snp, torch, cfg, scene, cams, targets, params, tg, n_norm, grad_ref)
        log(f"[bench] oracle gradient check: {grad_check}")

    # ---- Adam over every parameter (HBM bound; after the step, not in the metric) --
    optimizer = adam_leg(snp, torch, params)
    log(f"[bench] adam: {optimizer}")
    extras = training_extras_leg(snp, torch, cfg, scene, cams, params, tg, n_norm)
    log(f"[bench] training extras: {extras}")

    # ---- per-view plain launches ---------------------------------------------------------
    per_view_ms = None
    per_view_equal = None
    if not a.no_per_view:
        per_view_ms, per_view_equal = per_view_leg(snp, torch, cfg, scene, cams, params, tg, n_norm, img_batched, a)
        log(f"[bench] per-view plain launches: {per_view_ms:.3f} ms/step, images identical: {per_view_equal}")

    # ---- roofline of the dominant kernel ----------------------------------------------------
    ops = ops_per_pair(N, scene["cmlp_width"] if scene["color_mode"] == 4 else 0)

    def bwd_slots_of(cached_fraction):
        hit = hit_pairs * (cached_fraction * slots(ops["bwd_hit_cached"]) + (1 - cached_fraction) * slots(ops["bwd_hit"]))
        return hit + live_pairs * slots(ops["bwd_live"])

    fwd_slots = hit_pairs * slots(ops["fwd"])
    bwd_slots = bwd_slots_of(cached_frac)
    if bwd_ms >= fwd_ms:
        dom, dom_ms, dom_slots = "render_bwd", bwd_ms, bwd_slots
    else:
        dom, dom_ms, dom_slots = "render_fwd", fwd_ms, fwd_slots
    achieved = dom_slots / (dom_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3), "peak": round(PEAK_SLOTS / 1e12, 3),
                "unit": "Tslot/s", "frac": round(achieved / (PEAK_SLOTS / 1e12), 4),
                "traffic": measured_traffic(a.workload, dom, pair_cache),
                "kernel_ms": round(dom_ms, 4),
                "fwd_frac": round(fwd_slots / (fwd_ms * 1e-3) / PEAK_SLOTS, 4),
                "bwd_frac": round(bwd_slots / (bwd_ms * 1e-3) / PEAK_SLOTS, 4),
                "fwd_bwd_frac": round((fwd_slots + bwd_slots) / ((fwd_ms + bwd_ms) * 1e-3) / PEAK_SLOTS, 4),
                "slots_per_pair": {"fwd_hit": slots(ops["fwd"]), "bwd_hit_cached": slots(ops["bwd_hit_cached"]),
                                   "bwd_hit_recomputed": slots(ops["bwd_hit"]), "bwd_live": slots(ops["bwd_live"])}}
    if recompute is not None:
        rb = bwd_slots_of(0.0)
        recompute["bwd_frac"] = round(rb / (recompute["bwd_ms"] * 1e-3) / PEAK_SLOTS, 4)
        recompute["fwd_frac"] = round(fwd_slots / (recompute["fwd_ms"] * 1e-3) / PEAK_SLOTS, 4)

    value = hit_pairs / (ms_step * 1e-3)
    out = {
        "metric": "fwd+bwd pixel-primitive pairs/s; batched vs per-view ms/step @1e-4 img err",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded primitives, random-pose cameras, random targets)",
        "config": {"workload": workload_name(a.workload, cams), "primitives": scene["P"], "n_hidden": N,
                   "colour_mlp": [scene["cmlp_width"], scene["cmlp_depth"]], "tile": list(tile),
                   "batched": "one HIP graph per step, persistent rasterizer launches",
                   "pair_cache": pair_cache, "pair_cache_gib": round(cache_gb, 2),
                   "pair_cache_instances_frac": round(cached_frac, 4)},
        "hit_pairs_per_step": hit_pairs,
        "live_pairs_per_step": live_pairs,
        "instances_per_step": inst,
        "status_ok": status_ok,
        "max_img_err": None if check is None else check["max_img_err"],
        "oracle_check": check,
        "per_view_ms_per_step": per_view_ms,
        "batched_speedup_vs_per_view": (per_view_ms / ms_step) if per_view_ms else None,
        "per_view_images_identical": per_view_equal,
        "raster_fwd_ms": fwd_ms,
        "raster_bwd_ms": bwd_ms,
        "without_pair_cache": recompute,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "oracle_grad_check": grad_check,
        "optimizer": optimizer,
        "training_extras": extras,
        "paper_context": "218.87 FPS forward-only full pipeline, 100k random primitives, RTX 4090 (App. A)",
    }
    print(json.dumps(out))


def eager_kernel_ms(snp, rmod, torch, rast, params, images, final_T, tg, n_norm, steps):
    """Mean forward and backward rasterizer kernel times (ms) over a few
    eager steps, from the HIP events the library records on the launch
    stream around each launch."""
    rmod.kernel_timing(True)
    fwd_ms, bwd_ms = [], []
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    dL = torch.empty_like(images)
    grads = snp.zeros_like_params(params)
    rast.step(params, images, final_T, tg, n_norm, loss, dL, grads)
    for _ in range(max(3, min(steps, 5))):
        rast.step(params, images, final_T, tg, n_norm, loss, dL, grads)
        f, b = rmod.kernel_timing_read()
        fwd_ms.append(f)
        bwd_ms.append(b)
    rmod.kernel_timing(False)
    rast.read_status()
    return float(np.mean(fwd_ms)), float(np.mean(bwd_ms))


def adam_leg(snp, torch, params):
    """One Adam step over every parameter group (one launch), timed."""
    from paper_2510_08491_amd import train as TR
    grads = {k: torch.randn_like(v) * 1e-3 for k, v in params.items() if k in TR.PAPER_LRS}
    opt_params = {k: v.clone() for k, v in params.items() if k in TR.PAPER_LRS}
    opt = TR.Adam(opt_params)
    n_elems = sum(v.numel() for v in opt_params.values())
    opt.step(grads)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        opt.step(grads)
    e1.record()
    torch.cuda.synchronize()
    adam_ms = e0.elapsed_time(e1) / 5
    adam_bytes = 28 * n_elems  # read param, grad, m, v; write param, m, v (float32)
    del opt, opt_params, grads
    torch.cuda.empty_cache()
    return {"kernel": "adam (all groups, one launch)", "ms": round(adam_ms, 4), "elements": n_elems,
            "bytes": adam_bytes, "GB_per_s": round(adam_bytes / (adam_ms * 1e-3) / 1e9, 1),
            "frac_of_hbm_peak": round(adam_bytes / (adam_ms * 1e-3) / 8e12, 4)}


def training_extras_leg(snp, torch, cfg, scene, cams, params, tg, n_norm):
    """The other training-step kernels on this scene, timed after one
    gradient step (not in the metric): the scale regulariser, the
    population-control statistic and one population-control pass (plan on
    the device, one synchronisation for the new count, rows carried over
    with their two Adam moments)."""
    from paper_2510_08491_amd import train as TR
    r = snp.Rasterizer(snp.RenderConfig(**{**cfg.__dict__, "fwd_cache": 0}), scene["P"], cams)
    r._alloc(int(r.prepare(params) * 1.1) + 4096)
    images, T = r.new_images()
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    dL = torch.empty_like(images)
    grads = snp.zeros_like_params(params)
    r.step(params, images, T, tg, n_norm, loss, dL, grads)
    P = scene["P"]
    acc = torch.zeros(P, dtype=torch.float32, device="cuda")
    vis = torch.zeros(P, dtype=torch.float32, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    reg_ms = timed(lambda: TR.scale_regularizer(r, params["scales"], 0.01, grad_scales=grads["scales"]))
    acc_ms = timed(lambda: TR.densify_accumulate(r, grads, acc, vis))
    N = scene["N"]
    reg_bytes = 36 * P                                    # scales read, scale gradients read and written
    acc_bytes = (4 * (5 * N + 1) + 4 * len(cams) + 16) * P  # density-MLP gradients, tile counts, statistic
    keys = [k for k in params if k in TR.PAPER_LRS or k in ("w1", "b1", "w2", "b2")]
    pp = {k: params[k].clone() for k in keys}
    state = {f"{m}_{k}": torch.zeros_like(pp[k]) for k in keys for m in ("m", "v")}
    noise = torch.randn(P, 2, 3, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    new_p, _, action = TR.densify(pp, state, acc, vis, noise)
    torch.cuda.synchronize()
    dens_ms = 1e3 * (time.perf_counter() - t0)
    n_new = int(new_p["centers"].shape[0])
    del r, images, T, dL, grads, pp, state, new_p, action, acc, vis, noise
    torch.cuda.empty_cache()
    return {"scale_regularizer": {"ms": round(reg_ms, 4), "bytes": reg_bytes,
                                  "GB_per_s": round(reg_bytes / (reg_ms * 1e-3) / 1e9, 1)},
            "densify_statistic": {"ms": round(acc_ms, 4), "bytes": acc_bytes,
                                  "GB_per_s": round(acc_bytes / (acc_ms * 1e-3) / 1e9, 1)},
            "densify_pass": {"ms_wall": round(dens_ms, 3), "primitives_before": P, "primitives_after": n_new,
                             "note": "plan with the default thresholds on the statistic of the six timed accumulations "
                                     "(most primitives of the random scene fall under the prune threshold), one host "
                                     "synchronisation, allocation of the new arrays, row carry-over"}}


def per_view_leg(snp, torch, cfg, scene, cams, params, tg, n_norm, img_batched, a):
    """The same step as V separate pipelines of plain launches (one camera
    each, no graph, no persistent grid, the same kernels and tile shape).
    Returns (ms per step, images bitwise equal to the batched ones)."""
    cfg_pv = snp.RenderConfig(**{**cfg.__dict__, "persistent": 0})
    rv = []
    for c in cams:
        r = snp.Rasterizer(cfg_pv, scene["P"], [c])
        r._alloc(int(r.prepare(params) * 1.1) + 4096)
        rv.append(r)
    offs = np.cumsum([0] + [c.width * c.height for c in cams])
    outs = [r.new_images() for r in rv]
    dls = [torch.empty_like(o[0]) for o in outs]
    losses = [torch.zeros(1, dtype=torch.float64, device="cuda") for _ in rv]
    pv_grads = snp.zeros_like_params(params)

    def per_view_step():
        for g in pv_grads.values():
            g.zero_()
        for v, r in enumerate(rv):
            r.preprocess(params)
            r.bin()
            r.sort()
            r.forward(params, outs[v][0], outs[v][1])
            r.loss_l1(outs[v][0], tg[3 * offs[v]:3 * offs[v + 1]], n_norm, losses[v], dls[v])
            r.backward(params, outs[v][0], dls[v], pv_grads)

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(a.warmup):
        per_view_step()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(a.steps):
        per_view_step()
    e1.record()
    torch.cuda.synchronize()
    for r in rv:
        r.read_status()
    ms = e0.elapsed_time(e1) / a.steps
    equal = all(torch.equal(outs[v][0], img_batched[3 * offs[v]:3 * offs[v + 1]]) for v in range(len(cams)))
    del rv, outs, dls
    torch.cuda.empty_cache()
    return ms, bool(equal)


def oracle_check(scene, cams, cfg, images, tile_pairs, max_views, per_view=1):
    """`per_view` tiles per view (up to max_views views, spread over the
    list), chosen by a seeded draw without replacement among the tiles whose
    oracle instance count is at least the view's median (the deep lists):
    the oracle renders each tile's window in float64
    (oracle.render.render_window), compared with the batched step's image
    there and with the GPU's hit-pair count of that tile.  Returns the
    largest image error and both pair totals."""
    from oracle.keys import project_all
    from oracle.render import RenderOptions, render_window

    opts = RenderOptions(z_near=cfg.z_near, t_eps=cfg.t_eps, alpha_min=cfg.alpha_min, alpha_max=cfg.alpha_max,
                         bg=tuple(cfg.bg))
    rng = np.random.default_rng(4)
    img = images.cpu().numpy()
    V = len(cams)
    views = sorted(set(np.linspace(0, V - 1, min(V, max_views)).round().astype(int).tolist()))
    tw, th = cfg.tile_w, cfg.tile_h
    pix_off = np.cumsum([0] + [c.width * c.height for c in cams])
    tile_off = np.cumsum([0] + [((c.width + tw - 1) // tw) * ((c.height + th - 1) // th) for c in cams])
    t0 = time.perf_counter()
    worst, gpu_pairs, ora_pairs, npix, eq = 0.0, 0, 0, 0, True
    picked = []
    for v in views:
        cam = cams[v]
        proj = project_all(scene, cam, tw, th, cfg.z_near)
        ntx, nty = (cam.width + tw - 1) // tw, (cam.height + th - 1) // th
        # instances per tile from the oracle's tile rectangles (2-D difference array)
        tr = proj["trect"][proj["nonempty"]]
        diff = np.zeros((nty + 1, ntx + 1), np.int64)
        np.add.at(diff, (tr[:, 2], tr[:, 0]), 1)
        np.add.at(diff, (tr[:, 2], tr[:, 1] + 1), -1)
        np.add.at(diff, (tr[:, 3] + 1, tr[:, 0]), -1)
        np.add.at(diff, (tr[:, 3] + 1, tr[:, 1] + 1), 1)
        counts = diff.cumsum(0).cumsum(1)[:nty, :ntx].ravel()
        cand = np.nonzero(counts >= max(1, np.median(counts)))[0]
        view_img = img[3 * pix_off[v]:3 * pix_off[v + 1]].reshape(cam.height, cam.width, 3)
        chosen = rng.choice(cand, size=min(per_view, len(cand)), replace=False) if per_view > 1 else [rng.choice(cand)]
        for t in chosen:
            t = int(t)
            ty, tx = divmod(t, ntx)
            x0, y0 = tx * tw, ty * th
            w, h = min(tw, cam.width - x0), min(th, cam.height - y0)
            ref = render_window(scene, cam, x0, y0, w, h, opts, proj=proj)
            err = float(np.max(np.abs(view_img[y0:y0 + h, x0:x0 + w] - ref["image"])))
            worst = max(worst, err)
            gp = int(tile_pairs[tile_off[v] + t])
            gpu_pairs += gp
            ora_pairs += int(ref["hit_pairs"])
            eq = eq and gp == int(ref["hit_pairs"])
            npix += w * h
            picked.append([int(v), int(t), int(ref["primitives"])])
    return {"views": len(views), "tiles": len(picked), "pixels": npix, "max_img_err": worst,
            "hit_pairs_gpu": gpu_pairs, "hit_pairs_oracle": ora_pairs, "hit_pairs_equal": bool(eq),
            "tiles_view_tile_primitives": picked, "seconds": round(time.perf_counter() - t0, 1)}


_GRAD_SCENE = None  # the scene the gradient-check workers slice (inherited through fork)


def _grad_window(job):
    """One window of the gradient check: the oracle's autograd gradient of
    the L1 loss over the window, with respect to primitive `p`, scaled by the
    window's share of the loss's pixel count; and the signs of the oracle's
    image minus the target there."""
    import torch
    from oracle.grad import autograd_loss_and_grads
    from oracle.render import window_camera
    torch.set_num_threads(1)
    ids, i, cam, x0, y0, w, h, tgt, opts, n_norm = job
    scene = _GRAD_SCENE
    sub = dict(scene)
    for k, val in scene.items():
        if isinstance(val, np.ndarray) and val.ndim >= 1 and val.shape[0] == scene["P"]:
            sub[k] = val[ids]
    sub["P"] = len(ids)
    _, g, wimg = autograd_loss_and_grads(sub, [window_camera(cam, x0, y0, w, h)], [tgt], opts)
    return {k: v[i] * (w * h * 3 / n_norm) for k, v in g.items()}, np.sign(wimg[0] - tgt)


def oracle_grad_reference(scene, cams, targets, K):
    """The oracle's side of the gradient check, on the host before the GPU
    is touched (its workers are forked): K primitives drawn (seeded) among
    the quarter with the smallest footprints; a primitive changes only the
    pixels inside its rectangle, so its exact gradient is the sum over the
    views of the gradient of the L1 loss restricted to its rectangle there,
    rendered with every primitive that meets the rectangle (in index order,
    so the depth order is kept).  Returns the primitives, their reference
    gradients, and per window the oracle's signs of image minus target."""
    import multiprocessing as mp
    from oracle.keys import project_all
    from oracle.render import RenderOptions
    from paper_2510_08491_amd.render import RenderConfig

    global _GRAD_SCENE
    cfg = RenderConfig()
    opts = RenderOptions(z_near=cfg.z_near, t_eps=cfg.t_eps, alpha_min=cfg.alpha_min, alpha_max=cfg.alpha_max,
                         bg=tuple(cfg.bg))
    t0 = time.perf_counter()
    P = scene["P"]
    n_norm = float(sum(np.asarray(t).size for t in targets))
    projs = [project_all(scene, c, 16, 16, cfg.z_near) for c in cams]
    area = np.zeros(P)
    for pr in projs:
        rr = pr["rect"]
        area += np.where(pr["nonempty"], (rr[:, 1] - rr[:, 0] + 1) * (rr[:, 3] - rr[:, 2] + 1), 0)
    cand = np.nonzero((area > 0) & (area <= np.quantile(area[area > 0], 0.25)))[0]
    picked = np.sort(np.random.default_rng(5).choice(cand, size=min(K, len(cand)), replace=False))
    jobs, where = [], []
    for p in picked:
        for v, cam in enumerate(cams):
            pr = projs[v]
            if not pr["nonempty"][p]:
                continue
            x0, x1, y0, y1 = (int(x) for x in pr["rect"][p])
            rr = pr["rect"]
            ids = np.nonzero(pr["nonempty"] & (rr[:, 0] <= x1) & (rr[:, 1] >= x0) & (rr[:, 2] <= y1)
                             & (rr[:, 3] >= y0))[0]
            jobs.append((ids, int(np.searchsorted(ids, p)), cam, x0, y0, x1 - x0 + 1, y1 - y0 + 1,
                         targets[v][y0:y1 + 1, x0:x1 + 1], opts, n_norm))
            where.append((int(p), v, x0, y0, x1 - x0 + 1, y1 - y0 + 1))
    _GRAD_SCENE = scene
    res = []
    with mp.get_context("fork").Pool(host_cores()) as pool:
        for r in pool.imap(_grad_window, jobs, chunksize=1):
            res.append(r)
            if len(res) % 16 == 0:
                log(f"[bench] oracle gradient windows: {len(res)} of {len(jobs)}")
    ref = {}
    for (p, *_), (g, _) in zip(where, res):
        acc = ref.setdefault(p, {})
        for k, v in g.items():
            acc[k] = acc.get(k, 0.0) + v
    windows = [(w, sg) for w, (_, sg) in zip(where, res)]
    return {"primitives": [int(p) for p in picked], "ref": ref, "windows": windows,
            "seconds": round(time.perf_counter() - t0, 1)}


def oracle_grad_check(snp, torch, cfg, scene, cams, targets, params, tg, n_norm, reference):
    """The GPU's side: gradients from one step of the bench's own launch
    (configuration, tile, pair cache) for the reference's primitives, each
    parameter array compared normwise with the oracle's; and the window
    pixels where the GPU's image and the oracle's fall on different sides of
    the target (the L1 gradients' signs differ there, so the comparison
    would not hold)."""
    r = snp.Rasterizer(cfg, scene["P"], cams)
    r._alloc(int(r.prepare(params) * 1.1) + 4096)
    images, T = r.new_images()
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    dL = torch.empty_like(images)
    grads = snp.zeros_like_params(params)
    r.step(params, images, T, tg, n_norm, loss, dL, grads)
    torch.cuda.synchronize()
    img = images.cpu().numpy()
    del r, images, T, dL
    torch.cuda.empty_cache()
    pix_off = np.cumsum([0] + [c.width * c.height for c in cams])
    flips, wpix = {}, 0
    for (p, v, x0, y0, w, h), sg in reference["windows"]:
        cam = cams[v]
        gimg = img[3 * pix_off[v]:3 * pix_off[v + 1]].reshape(cam.height, cam.width, 3)[y0:y0 + h, x0:x0 + w]
        flips[p] = flips.get(p, 0) + int(np.sum(np.sign(gimg - targets[v][y0:y0 + h, x0:x0 + w]) != sg))
        wpix += w * h
    # primitives whose windows hold a pixel of opposite loss-gradient sign are
    # reported but not compared
    clean = [p for p in reference["ref"] if flips.get(p, 0) == 0]
    diff, scale, worst_p = {}, {}, {}
    for p in clean:
        for k, rk in reference["ref"][p].items():
            if k not in grads:
                continue
            gg = grads[k][int(p)].detach().cpu().numpy().astype(np.float64)
            d, m = float(np.max(np.abs(gg - rk))), float(np.max(np.abs(rk)))
            diff[k], scale[k] = max(diff.get(k, 0.0), d), max(scale.get(k, 0.0), m)
            worst_p[k] = max(worst_p.get(k, 0.0), d / m if m > 0 else d)
    return {"primitives": reference["primitives"], "windows": len(reference["windows"]), "window_pixels": wpix,
            "sign_flip_pixels": {str(p): n for p, n in flips.items() if n},
            "compared": len(clean),
            # max |g - g_ref| over the compared primitives / max |g_ref| (reading of the tolerance: normwise)
            "normwise_err": {k: float(f"{diff[k] / scale[k]:.3g}") for k in diff if scale[k] > 0},
            # the same per primitive, the worst one
            "worst_per_primitive_err": {k: float(f"{e:.3g}") for k, e in worst_p.items()},
            "oracle_seconds": reference["seconds"]}


def _fps(snp, torch, scene, cams, cfg, a, label):
    """Frames/s of the forward pipeline (preprocess, bin, sort, render) with
    one view per pipeline (frames one after another over the views) and with
    all views in one batched pipeline.  Also the render kernel's own time per
    frame (library events, an untimed pass) and the hit pairs per frame."""
    params = snp.params_to_device(scene)
    rasts, outs, pairs = [], [], 0
    for c in cams:
        r = snp.Rasterizer(cfg, scene["P"], [c])
        r._alloc(int(r.prepare(params) * 1.1) + 4096)
        r.prepare(params)
        img, T = r.new_images()
        r.forward(params, img, T, count_pairs=True)
        pairs += r.counters()["hit_pairs"]
        rasts.append(r)
        outs.append((img, T))

    def frame(i):
        # the stages without the host round trip of prepare()'s capacity
        # check (the device still flags an overflow; it is read after the
        # timed frames)
        r = rasts[i % len(rasts)]
        r.preprocess(params)
        r.bin()
        r.sort()
        r.forward(params, *outs[i % len(rasts)])

    for i in range(max(a.warmup, 1) * len(rasts)):
        frame(i)
    torch.cuda.synchronize()
    n = max(a.steps, 1) * len(rasts)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(n):
        frame(i)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / n
    for r in rasts:
        r.read_status()  # raises if any frame overflowed its workspace
    # the same frames replayed from one captured forward graph per view
    graphs = [snp.ForwardGraph(r, params, *o) for r, o in zip(rasts, outs)]
    for i in range(max(a.warmup, 1) * len(graphs)):
        graphs[i % len(graphs)].launch()
    torch.cuda.synchronize()
    e0.record()
    for i in range(n):
        graphs[i % len(graphs)].launch()
    e1.record()
    torch.cuda.synchronize()
    ms_g = e0.elapsed_time(e1) / n
    for r in rasts:
        r.read_status()
    del graphs
    snp.kernel_timing(True)
    kms = []
    for i in range(len(rasts)):
        frame(i)
        kms.append(snp.kernel_timing_read()[0])
    snp.kernel_timing(False)
    render_ms = sum(kms) / len(kms)
    log(f"[bench] {label}: hit pairs per frame {pairs / len(cams):.4g}; one view per pipeline: {ms:.3f} ms/frame, "
        f"{1e3 / ms:.1f} frames/s plain launches, {ms_g:.3f} ms/frame, {1e3 / ms_g:.1f} frames/s graph replays "
        f"(render kernel {render_ms:.3f} ms)")
    rb = snp.Rasterizer(cfg, scene["P"], cams)
    rb._alloc(int(rb.prepare(params) * 1.1) + 4096)
    img_b, T_b = rb.new_images()
    for _ in range(max(a.warmup, 1)):
        rb.prepare(params)
        rb.forward(params, img_b, T_b)
    torch.cuda.synchronize()
    nb = max(a.steps, 1)
    e0.record()
    for _ in range(nb):
        rb.preprocess(params)
        rb.bin()
        rb.sort()
        rb.forward(params, img_b, T_b)
    e1.record()
    torch.cuda.synchronize()
    rb.read_status()
    ms_b = e0.elapsed_time(e1) / (nb * len(cams))
    offs = np.cumsum([0] + [3 * c.width * c.height for c in cams])
    same = all(torch.equal(outs[v][0], img_b[offs[v]:offs[v + 1]]) for v in range(len(cams)))
    log(f"[bench] {label}: all views in one pipeline: {ms_b:.3f} ms/frame, {1e3 / ms_b:.1f} frames/s, "
        f"images identical: {same}")
    del rasts, outs, rb
    torch.cuda.empty_cache()
    return dict(ms=ms, ms_g=ms_g, ms_b=ms_b, render_ms=render_ms, pairs=pairs / len(cams), same=same)


def forward_fps(a):
    """Forward-only throughput on the stand-in for the paper's App. A protocol
    (100k random primitives in a volume, N = 8, omega0 = 30, degree-3 SH
    colour, 800x800 views), and the same scene as Gaussian splats (the 3DGS
    kernel the paper compares against): every frame runs the whole forward
    pipeline for one view; reports frames/s of both and their ratio."""
    import torch
    import paper_2510_08491_amd as snp
    import synthetic as S
    _, scene, cams, _ = S.make_workload("A")
    tile = tuple(int(x) for x in a.tile.split(",")) if a.tile else (16, 16, 1)
    cfg = snp.RenderConfig(n_hidden=scene["N"], omega0=scene["omega0"], color_mode=scene["color_mode"],
                           bin_order=a.bin_order,
                           tile_w=tile[0], tile_h=tile[1], px_per_lane=tile[2], persistent=1, fwd_cache=0)
    log(f"[bench] workload A: P={scene['P']} views={len(cams)} {cams[0].width}x{cams[0].height} "
        f"N={scene['N']} tile={tile}")
    nn = _fps(snp, torch, scene, cams, cfg, a, "neural primitives")
    _, gscene, gcams, _ = S.make_workload("G")
    gcfg = snp.RenderConfig(color_mode=gscene["color_mode"], primitive=1, bin_order=a.bin_order, tile_w=tile[0],
                            tile_h=tile[1],
                            px_per_lane=tile[2], persistent=1, alpha_min=1.0 / 255.0)
    gs = _fps(snp, torch, gscene, gcams, gcfg, a, "Gaussians")
    ms, ms_b = nn["ms"], nn["ms_b"]
    out = {
        "metric": "forward frames/s, full pipeline (preprocess, bin, sort, render) per view",
        "value": 1e3 / ms, "unit": "frames/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded primitives, random-pose cameras)",
        "config": {"workload": f"{scene['P']} random primitives in [-1,1]^3, N={scene['N']}, omega0={scene['omega0']}, "
                               f"degree-3 SH colour, {len(cams)} views of {cams[0].width}x{cams[0].height}, forward only",
                   "tile": list(tile)},
        "hit_pairs_per_frame": nn["pairs"],
        "pairs_per_s": nn["pairs"] / (ms * 1e-3),
        "render_kernel_ms": nn["render_ms"],
        "graph_replay_frames_per_s": 1e3 / nn["ms_g"],
        "batched_frames_per_s": 1e3 / ms_b,
        "batched_images_identical": nn["same"],
        "gaussians": {"workload": "the same primitives as 3D Gaussians (standard deviations a third of the scales, "
                                  "opacity U(0.2, 0.9), alpha_min 1/255)",
                      "frames_per_s": 1e3 / gs["ms"], "graph_replay_frames_per_s": 1e3 / gs["ms_g"],
                      "batched_frames_per_s": 1e3 / gs["ms_b"],
                      "render_kernel_ms": gs["render_ms"], "hit_pairs_per_frame": gs["pairs"],
                      "batched_images_identical": gs["same"]},
        "gaussian_over_neural_fps": nn["ms"] / gs["ms"],
        "paper_context": "App. A, RTX 4090: 218.87 FPS for 100k random neural primitives, 546.54 FPS for 3DGS "
                         "(ratio 2.50) on synthetic-NeRF cameras; primitive sizes there are not given, so the "
                         "absolute rates are not comparable one to one",
    }
    print(json.dumps(out))


def measured_traffic(workload, kernel, pair_cache):
    """HBM bytes per launch of `kernel` from the rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary in profiles/ (scaled by a copy kernel of known size),
    or None when there is none for this workload and pair-cache mode, or the
    rasterizer source has changed since the counters were taken."""
    import hashlib
    suffix = "" if pair_cache else "_recompute"
    path = os.path.join(ROOT, "profiles", f"{workload.lower()}_render_traffic{suffix}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        parts = line.split()
        if len(parts) == 2 and parts[0] in ("source_sha256", "render_bwd_bytes", "render_fwd_bytes"):
            vals[parts[0]] = parts[1]
    csrc = os.path.join(ROOT, "paper_2510_08491_amd", "csrc")
    src = open(os.path.join(csrc, "raster.hip"), "rb").read() + open(os.path.join(csrc, "snp_internal.h"), "rb").read()
    if vals.get("source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    key = {"render_bwd": "render_bwd_bytes", "render_fwd": "render_fwd_bytes"}[kernel]
    return float(vals[key]) if key in vals else None


def workload_name(w, cams):
    sizes = {}
    for c in cams:
        sizes[f"{c.width}x{c.height}"] = sizes.get(f"{c.width}x{c.height}", 0) + 1
    desc = " + ".join(f"{n}x{k}" for k, n in sizes.items())
    return {"C3": "1 camera 1920x1080, 200k primitives, N=16, colour MLP W32 D2, fwd+bwd",
            "C4": f"16 mixed cameras ({desc}), 200k primitives, N=16, colour MLP W32 D2, batched fwd+bwd",
            "C5": "32 cameras 1600x900, 1M primitives, N=32, colour MLP W32 D3, batched fwd+bwd",
            "R": f"16 mixed cameras ({desc}), 200k primitives, N=16, per-ray relighting colour network W16 D1 "
                 "with a point light per view, batched fwd+bwd",
            "L": f"16 mixed cameras ({desc}), 200k primitives, N=16, relighting colour network W32 D2 per "
                 "(primitive, view) with a point light per view, batched fwd+bwd",
            "D": f"16 mixed cameras ({desc}), 200k primitives, N=16, time-conditioned density and degree-3 SH "
                 "colour with the time-dependent zero-order coefficient at xi_t=0.5, batched fwd+bwd"}[w]


def _oracle_crop(job):
    """One crop: the FP64 oracle's forward (numpy) and its autograd backward
    (torch float64) on the primitives that touch the crop.  Returns (hit
    pairs, seconds)."""
    import torch
    from oracle.grad import autograd_loss_and_grads
    from oracle.render import RenderOptions, render_view
    torch.set_num_threads(1)
    sub, crop, tgt = job
    t0 = time.perf_counter()
    r = render_view(sub, crop, RenderOptions())
    autograd_loss_and_grads(sub, [crop], tgt, RenderOptions())
    return r["hit_pairs"], time.perf_counter() - t0


def host_cores():
    """The cores this process may run on, at most 16 (one GPU's share of
    the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(scene, cams, targets, budget_s, workload):
    """The FP64 oracle (numpy forward + torch float64 autograd backward) on
    16x16-pixel crops of the workload's views, each with the primitives whose
    screen bounds touch it (the only ones that contribute to it; selecting
    them is not timed), one crop per worker process at a time over the
    host's cores; about `budget_s` seconds of wall time.  Returns hit pairs
    per wall-clock second.  Also times the 64x64, 256-primitive scene's
    whole forward + backward in one process."""
    import multiprocessing as mp
    import synthetic as S
    from oracle.keys import project_all

    cores = host_cores()
    rng = np.random.default_rng(3)
    size = 16

    def make_job():
        v = int(rng.integers(0, len(cams)))
        cam = cams[v]
        x0 = int(rng.integers(cam.width // 4, 3 * cam.width // 4 - size))
        y0 = int(rng.integers(cam.height // 4, 3 * cam.height // 4 - size))
        crop = S.Camera(size, size, cam.fx, cam.fy, cam.cx - x0, cam.cy - y0, cam.R, cam.t)
        ids = np.nonzero(project_all(scene, crop)["nonempty"])[0]
        return S.subset_scene(scene, ids), crop, [targets[v][y0:y0 + size, x0:x0 + size]]

    # calibrate the crop count on one crop, then run them all in the pool;
    # the calibration runs in a child too: a process that has run an
    # autograd backward cannot fork workers that run one
    ctx = mp.get_context("fork")
    probe = make_job()
    with ctx.Pool(1) as pool:
        pairs0, sec0 = pool.apply(_oracle_crop, (probe,))
    n_jobs = max(cores, int(round(budget_s / max(sec0, 1e-3))) * cores)
    n_jobs = min(n_jobs, 8 * cores)
    jobs = [make_job() for _ in range(n_jobs)]
    prims = sum(j[0]["P"] for j in jobs)
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_crop, jobs, chunksize=1)
    wall = time.perf_counter() - t0
    pairs = sum(r[0] for r in res)
    busy = sum(r[1] for r in res)
    # the smallest workload, whole: 64x64, 256 primitives, N = 8, constant colour
    _, s1, c1, t1 = S.make_workload("C1")
    p1, sec1 = _oracle_crop((s1, c1[0], t1))
    return {"value": pairs / wall, "unit": "pairs/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_jobs} random {size}x{size} px crops of the central half of random views of the "
                      f"{workload} workload, each with the primitives whose bounds touch it "
                      f"({prims // max(n_jobs, 1)} on average of {scene['P']}); FP64 numpy forward + torch "
                      f"float64 autograd backward; {cores} worker processes (one thread each, "
                      f"{busy / wall:.1f} busy on average); {pairs} hit pairs in {wall:.1f} s wall",
            "c1_full_fwd_bwd": {"seconds": round(sec1, 3), "hit_pairs": int(p1), "pairs_per_s": p1 / sec1,
                                "threads": 1}}


if __name__ == "__main__":
    main()
