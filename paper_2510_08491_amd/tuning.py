"""Autotuner for the rasterizer's launch shape.

For a workload class (density width N, colour mode, resolution class of the
cameras) it times every tile shape the library is built for -- tile width,
tile height and pixels per thread -- on a real forward + backward, checks
that every candidate renders the same image as the first, and stores the
fastest in a JSON cache next to this file.  `lookup` reads the cache.
"""
from __future__ import annotations

import ctypes as C
import json
import os
from typing import Dict, List, Optional, Tuple

import torch

from . import _lib as L
from .render import RenderConfig, Rasterizer, kernel_timing, kernel_timing_read, zeros_like_params

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")


def supported_shapes() -> List[Tuple[int, int, int]]:
    arr = (C.c_int32 * 96)()
    n = L.lib().snp_supported_tiles(arr, 32)
    return [tuple(arr[3 * i:3 * i + 3]) for i in range(n)]


def resolution_class(cams) -> str:
    px = sum(int(c.width) * int(c.height) for c in cams)
    return f"V{len(cams)}_MP{max(1, round(px / 1e6))}"


def key_of(N: int, color_mode: int, cams, fwd_cache: int = 1) -> str:
    """Workload class: density width, colour mode, resolution class, and
    whether the backward reads the forward's pair cache (the two backwards
    favour different batch sizes)."""
    arch = "gfx950"
    mode = "" if fwd_cache else "/recompute"
    return f"{arch}/N{N}/cm{color_mode}/{resolution_class(cams)}{mode}"


def _load() -> Dict:
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {}


def lookup(N: int, color_mode: int, cams, fwd_cache: int = 1) -> Optional[Tuple[int, int, int, int]]:
    """(tile_w, tile_h, px_per_lane, bwd_batch) tuned for this class, or None."""
    entry = _load().get(key_of(N, color_mode, cams, fwd_cache))
    if not entry:
        return None
    return tuple(entry["tile"]) + (int(entry.get("bwd_batch", 0)),)


def bwd_batches(base: RenderConfig, tw: int, th: int, cams) -> List[int]:
    """Backward batch sizes the library accepts for a tile shape (asked by
    validating a layout on the host)."""
    out = []
    for nb in (4, 8, 16, 32):
        cfg = RenderConfig(**{**base.__dict__, "tile_w": tw, "tile_h": th, "bwd_batch": nb})
        for ppl in (1, 2, 4):
            cfg.px_per_lane = ppl
            lay = L.SnpLayout()
            from .render import camera_array
            if L.lib().snp_workspace_layout(C.byref(cfg.to_c()), 1, len(cams), camera_array(cams), 1,
                                            C.byref(lay)) == L.SNP_OK:
                out.append(nb)
                break
    return out


def autotune(base: RenderConfig, P: int, cams, params, targets: torch.Tensor, reps: int = 2,
             shapes=None, write=True, log=print):
    """Times the rasterizer kernels for every tile shape, every forward
    pixels-per-thread count and every backward batch size (HIP events around
    the launches, best of `reps`); the forward time depends only on the
    former, the backward time only on the latter.  Checks that each candidate
    renders the same image as the first.  Returns (best (tile_w, tile_h,
    px_per_lane, bwd_batch), table)."""
    fwd_shapes = shapes or supported_shapes()
    tiles = sorted({(s[0], s[1]) for s in fwd_shapes})
    results = {}
    ref_img = None
    n_norm = float(targets.numel())
    best = None
    for tw, th in tiles:
        f_ppls = [s[2] for s in fwd_shapes if (s[0], s[1]) == (tw, th)]
        nbs = bwd_batches(base, tw, th, cams)
        runs = [(p, 0) for p in f_ppls] + [(f_ppls[0], nb) for nb in nbs]
        fwd_ms, bwd_ms = {}, {}
        for pf, nb in runs:
            cfg = RenderConfig(**{**base.__dict__, "tile_w": tw, "tile_h": th, "px_per_lane": pf, "bwd_batch": nb})
            rast = Rasterizer(cfg, P, cams)
            inst = rast.prepare(params)
            rast._alloc(int(inst * 1.1) + 4096)
            images, T = rast.new_images()
            loss = torch.zeros(1, dtype=torch.float64, device=images.device)
            dL = torch.empty_like(images)
            grads = zeros_like_params(params)
            rast.step(params, images, T, targets, n_norm, loss, dL, grads)   # warm-up
            kernel_timing(True)
            fb, bb = None, None
            for _ in range(reps):
                rast.step(params, images, T, targets, n_norm, loss, dL, grads)
                f, b = kernel_timing_read()
                fb = f if fb is None else min(fb, f)
                bb = b if bb is None else min(bb, b)
            kernel_timing(False)
            torch.cuda.synchronize()
            if ref_img is None:
                ref_img = images.clone()
            diff = float((images - ref_img).abs().max())
            if nb == 0:
                fwd_ms[pf] = fb
            else:
                bwd_ms[nb] = bb
            results[f"{tw}x{th} ppl{pf} batch{nb}"] = dict(fwd_ms=fb, bwd_ms=bb, img_diff=diff)
            log(f"[tune] tile {tw}x{th} ppl {pf} bwd batch {nb or 'default'}: forward {fb:.3f} ms, "
                f"backward {bb:.3f} ms, image diff {diff:.2e}")
            if diff > 1e-5:
                raise RuntimeError(f"tile {tw}x{th}/{pf} renders a different image ({diff})")
            del rast, images, T, dL, grads
            torch.cuda.empty_cache()
        pf = min(fwd_ms, key=fwd_ms.get)
        nb = min(bwd_ms, key=bwd_ms.get)
        total = fwd_ms[pf] + bwd_ms[nb]
        if best is None or total < best[0]:
            best = (total, (tw, th, pf, nb))
    best_shape = best[1]
    if write:
        cache = _load()
        cache[key_of(base.n_hidden, base.color_mode, cams, base.fwd_cache)] = {
            "tile": list(best_shape[:3]), "bwd_batch": best_shape[3], "ms": best[0], "candidates": results}
        with open(CACHE, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return best_shape, results


def main(argv=None):
    """python -m paper_2510_08491_amd.tuning --workload C4 [--out FILE]"""
    import argparse
    import sys

    import numpy as np

    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="C4")
    ap.add_argument("--out", default=None, help="also write the cache to this file")
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--fwd-cache", type=int, default=None, choices=[0, 1],
                    help="pair-cache mode to tune for (default: 0 for C5, else 1)")
    ap.add_argument("--shapes", default=None,
                    help="only these tile shapes, e.g. 16x16x1,32x16x2 (default: every built shape)")
    a = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import synthetic as S
    from .render import params_to_device

    _, scene, cams, targets = S.make_workload(a.workload)
    fwd_cache = a.fwd_cache if a.fwd_cache is not None else (0 if a.workload == "C5" else 1)
    base = RenderConfig(n_hidden=scene["N"], omega0=scene["omega0"], color_mode=scene["color_mode"],
                        cmlp_width=scene["cmlp_width"], cmlp_depth=scene["cmlp_depth"], persistent=1,
                        fwd_cache=fwd_cache)
    params = params_to_device(scene)
    tg = torch.from_numpy(np.concatenate([t.ravel() for t in targets])).cuda()
    shapes = None
    if a.shapes:
        shapes = [tuple(int(x) for x in sh.split("x")) for sh in a.shapes.split(",")]
    best, _ = autotune(base, scene["P"], cams, params, tg, reps=a.reps, shapes=shapes,
                       log=lambda m: print(m, flush=True))
    print(f"[tune] best tile for {key_of(base.n_hidden, base.color_mode, cams, fwd_cache)}: {best}", flush=True)
    if a.out:
        with open(CACHE) as f, open(a.out, "w") as g:
            g.write(f.read())


if __name__ == "__main__":
    main()
