"""Python side of the rasterizer: workspace management, the stage calls, a
torch.autograd.Function around forward/backward, and graph-captured batched
steps.  Everything numeric runs in libsnp (HIP); torch only provides device
memory and the stream."""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L

PARAM_KEYS = ("centers", "scales", "quats", "w1", "b1", "w2", "b2", "colors", "cmlp", "xi", "sh", "opacity", "wt",
              "sh_t")
XI_DIM = 8


@dataclasses.dataclass
class RenderConfig:
    n_hidden: int = 8
    omega0: float = 10.0
    color_mode: int = 0
    cmlp_width: int = 0
    cmlp_depth: int = 0
    tile_w: int = 16
    tile_h: int = 16
    px_per_lane: int = 1
    z_near: float = 0.2
    t_eps: float = 1e-4
    alpha_min: float = 0.0
    alpha_max: float = 0.99
    bg: tuple = (0.0, 0.0, 0.0)
    persistent: int = 0
    bwd_batch: int = 0
    # 1: the forward keeps every evaluated pair's integral for the backward
    # (tile pixels floats per instance) for as many leading instances as the
    # memory budget below holds, the backward re-evaluates the rest;
    # 0: the backward re-evaluates every pair
    fwd_cache: int = 1
    # device bytes the pair cache may take; None: 85% of the free memory
    # left after the rest of the workspace
    fwd_cache_budget: Optional[int] = None
    # 0 neural primitives; 1 Gaussian splats (forward only)
    primitive: int = 0
    # 1 depth sort of the (view, primitive) pairs then a tile-bit instance
    # sort; 2 one sort over all key bits; 0 picks by size (same result)
    bin_order: int = 0
    # xi_t of the time-conditioned density (used with a "wt" parameter)
    time: float = 0.0

    def to_c(self) -> L.SnpConfig:
        c = L.SnpConfig()
        for f in dataclasses.fields(self):
            if f.name == "fwd_cache_budget":
                continue
            if f.name == "bg":
                c.bg = (C.c_float * 3)(*self.bg)
            else:
                setattr(c, f.name, getattr(self, f.name))
        return c


def cmlp_param_count(width: int, depth: int, relight: bool = False, per_ray: bool = False) -> int:
    """Colour-network parameters per primitive: inputs view direction and
    xi (11), plus the light direction (14) for the relighting colour, or the
    entry point, ray direction and light direction (9) for the per-ray
    relighting colour."""
    if depth <= 0:
        return 0
    n_in = 9 if per_ray else (14 if relight else 11)
    return n_in * width + width + (depth - 1) * (width * width + width) + 3 * width + 3


def camera_array(cams) -> "C.Array":
    """Camera objects with width, height, fx, fy, cx, cy, R (3x3), t (3)
    -> a ctypes array of snp_camera."""
    arr = (L.SnpCamera * len(cams))()
    for i, c in enumerate(cams):
        a = arr[i]
        a.width, a.height = int(c.width), int(c.height)
        a.fx, a.fy, a.cx, a.cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
        a.R = (C.c_float * 9)(*np.asarray(c.R, np.float32).ravel().tolist())
        a.t = (C.c_float * 3)(*np.asarray(c.t, np.float32).ravel().tolist())
        light = getattr(c, "light", None)
        a.light = (C.c_float * 3)(*(np.zeros(3) if light is None else np.asarray(light, np.float32)).ravel().tolist())
    return arr


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous() and t.dtype == torch.float32, "float32 contiguous device tensors only"
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def params_to_device(scene: dict, device="cuda") -> Dict[str, torch.Tensor]:
    """numpy scene arrays (as from synthetic.make_scene) -> float32 device tensors."""
    out = {}
    for k in PARAM_KEYS:
        v = scene.get(k)
        if v is not None:
            out[k] = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).to(device)
    return out


class Rasterizer:
    """One workspace for P primitives seen by a fixed list of cameras."""

    def __init__(self, cfg: RenderConfig, P: int, cams, capacity: Optional[int] = None, device="cuda"):
        self.cfg = cfg
        self.ccfg = cfg.to_c()
        self.P = int(P)
        self.cams = list(cams)
        self.V = len(self.cams)
        self.ccams = camera_array(self.cams)
        self.device = device
        self.pixels = [int(c.width) * int(c.height) for c in self.cams]
        self.total_pixels = sum(self.pixels)
        self.layout = None
        self.ws = None
        # bumped by every call that rewrites the workspace (the stages, a
        # step, a graph replay, a re-allocation); a backward checks that the
        # workspace still holds the forward it differentiates
        self.generation = 0
        self._alloc(capacity if capacity is not None else max(1 << 16, 8 * self.P))

    # -- workspace ---------------------------------------------------------------
    def _layout(self, capacity: int, fwd_cache: int, cache_instances: int = 0) -> L.SnpLayout:
        self.ccfg.fwd_cache = int(fwd_cache)
        self.ccfg.fwd_cache_instances = int(cache_instances)
        lay = L.SnpLayout()
        L.check(L.lib().snp_workspace_layout(C.byref(self.ccfg), self.P, self.V, self.ccams, int(capacity),
                                             C.byref(lay)), "snp_workspace_layout")
        return lay

    def _alloc(self, capacity: int):
        self.generation += 1
        self.ws = None
        lay = self._layout(capacity, self.cfg.fwd_cache)
        if lay.ahat_cache_bytes:
            budget = self.cfg.fwd_cache_budget
            if budget is None:
                torch.cuda.empty_cache()  # the previous workspace is still held by the allocator's cache
                free, _ = torch.cuda.mem_get_info(torch.device(self.device))
                budget = int(0.85 * (free - (lay.bytes - lay.ahat_cache_bytes)))
            if lay.ahat_cache_bytes > budget:
                # cache the leading instances that fit; the backward re-evaluates the rest
                per_instance = lay.ahat_cache_bytes // int(capacity)
                n = max(0, budget) // per_instance
                lay = self._layout(capacity, 1, n) if n >= max(1, int(capacity) // 50) else self._layout(capacity, 0)
        self.layout = lay
        self.ws = torch.empty(lay.bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        self._ws_off = off
        self.ws_ptr = C.c_void_p(self.ws.data_ptr() + off)

    @property
    def capacity(self) -> int:
        return int(self.layout.capacity)

    @property
    def fwd_cache(self) -> bool:
        """True when the forward keeps pair integrals for the backward."""
        return bool(self.ccfg.fwd_cache)

    @property
    def cached_instances(self) -> int:
        """How many leading tile instances have their pair integrals kept."""
        if not self.ccfg.fwd_cache:
            return 0
        return int(self.layout.ahat_cache_bytes // (4 * self.cfg.tile_w * self.cfg.tile_h))

    def _view(self, field: str, dtype, count: int) -> torch.Tensor:
        start = self._ws_off + getattr(self.layout, field)
        nbytes = count * torch.empty((), dtype=dtype).element_size()
        return self.ws[start:start + nbytes].view(dtype)

    def keys(self, n):
        return self._view("keys", torch.int64, n)

    def values(self, n):
        return self._view("values", torch.int32, n)

    def ranges(self):
        return self._view("ranges", torch.int32, 2 * self.layout.total_tiles).view(-1, 2)

    def tile_pairs(self):
        """Hit pairs per global tile, counted by the last forward with
        count_pairs=True (tiles of view 0 first, row-major in each view)."""
        return self._view("tile_pairs", torch.int32, self.layout.total_tiles)

    def rects(self):
        return self._view("rects", torch.int32, 4 * self.V * self.P).view(self.V, self.P, 4)

    def depth_bits(self):
        return self._view("depth_bits", torch.int32, self.V * self.P).view(self.V, self.P)

    def tile_counts(self):
        return self._view("tile_counts", torch.int32, self.V * self.P).view(self.V, self.P)

    # -- stages --------------------------------------------------------------------
    def _prims(self, params) -> L.SnpPrims:
        pr = L.SnpPrims()
        pr.P = self.P
        for k in PARAM_KEYS:
            setattr(pr, k, _ptr(params.get(k)))
        return pr

    def preprocess(self, params):
        self.generation += 1
        L.check(L.lib().snp_preprocess(C.byref(self.ccfg), C.byref(self._prims(params)), self.V, self.ccams,
                                       self.ws_ptr, C.byref(self.layout), _stream()), "snp_preprocess")

    def bin(self):
        self.generation += 1
        L.check(L.lib().snp_bin(C.byref(self.ccfg), self.P, self.V, self.ccams, self.ws_ptr, C.byref(self.layout),
                                _stream()), "snp_bin")

    def sort(self):
        self.generation += 1
        L.check(L.lib().snp_sort(C.byref(self.ccfg), self.P, self.V, self.ccams, self.ws_ptr, C.byref(self.layout),
                                 _stream()), "snp_sort")

    def read_status(self, raise_on_error=True):
        inst, pairs = C.c_int64(0), C.c_int64(0)
        code = L.lib().snp_read_status(self.ws_ptr, C.byref(self.layout), C.byref(inst), C.byref(pairs), _stream())
        if raise_on_error and code not in (L.SNP_OK,):
            raise L.SnpError(code, "snp_read_status")
        return code, int(inst.value), int(pairs.value)

    def counters(self):
        """The 8 device counters (synchronises the stream)."""
        out = (C.c_int64 * 8)()
        L.check(L.lib().snp_read_counters(self.ws_ptr, C.byref(self.layout), out, _stream()), "snp_read_counters")
        return dict(instances=out[0], overflow=out[1], hit_pairs=out[2], range_flag=out[3], live_pairs=out[6])

    def prepare(self, params, grow=True):
        """preprocess + bin + sort; grows the workspace and redoes the stages
        if the tile instances overflowed it.  Returns the instance count."""
        while True:
            self.preprocess(params)
            self.bin()
            code, inst, _ = self.read_status(raise_on_error=False)
            if code == L.SNP_ERR_CAPACITY and grow:
                self._alloc(int(inst * 1.25) + 1024)
                continue
            if code != L.SNP_OK:
                raise L.SnpError(code, "prepare")
            break
        self.sort()
        return inst

    def new_images(self):
        img = torch.empty(3 * self.total_pixels, dtype=torch.float32, device=self.device)
        T = torch.empty(self.total_pixels, dtype=torch.float32, device=self.device)
        return img, T

    def forward(self, params, images, final_T, count_pairs=False):
        self.generation += 1
        L.check(L.lib().snp_render_forward(C.byref(self.ccfg), C.byref(self._prims(params)), self.V, self.ccams,
                                           self.ws_ptr, C.byref(self.layout), _ptr(images), _ptr(final_T),
                                           1 if count_pairs else 0, _stream()), "snp_render_forward")

    def loss_l1(self, images, targets, n_norm=None, loss_out=None, dL=None):
        n_norm = float(3 * self.total_pixels if n_norm is None else n_norm)
        loss_out = torch.zeros(1, dtype=torch.float64, device=self.device) if loss_out is None else loss_out
        dL = torch.empty_like(images) if dL is None else dL
        L.check(L.lib().snp_loss_l1(C.byref(self.ccfg), self.V, self.ccams, _ptr(images), _ptr(targets), n_norm,
                                    self.ws_ptr, C.byref(self.layout), C.c_void_p(loss_out.data_ptr()), _ptr(dL),
                                    _stream()), "snp_loss_l1")
        return loss_out, dL

    def grads_struct(self, grads: Dict[str, torch.Tensor]) -> L.SnpGrads:
        g = L.SnpGrads()
        for k, _ in L.SnpGrads._fields_:
            setattr(g, k, _ptr(grads.get(k)))
        return g

    def backward(self, params, images, dL, grads: Dict[str, torch.Tensor]):
        """Adds d loss / d params into `grads` (same keys/shapes as params)."""
        g = self.grads_struct(grads)
        L.check(L.lib().snp_render_backward(C.byref(self.ccfg), C.byref(self._prims(params)), self.V, self.ccams,
                                            self.ws_ptr, C.byref(self.layout), _ptr(images), _ptr(dL), C.byref(g),
                                            _stream()), "snp_render_backward")

    def step(self, params, images, final_T, targets, n_norm, loss_out, dL, grads):
        self.generation += 1
        g = self.grads_struct(grads)
        L.check(L.lib().snp_step(C.byref(self.ccfg), C.byref(self._prims(params)), self.V, self.ccams, self.ws_ptr,
                                 C.byref(self.layout), _ptr(images), _ptr(final_T), _ptr(targets), float(n_norm),
                                 C.c_void_p(loss_out.data_ptr()), _ptr(dL), C.byref(g), _stream()), "snp_step")

    def split_images(self, images: torch.Tensor) -> List[torch.Tensor]:
        out, off = [], 0
        for c, n in zip(self.cams, self.pixels):
            out.append(images[3 * off:3 * (off + n)].view(int(c.height), int(c.width), 3))
            off += n
        return out


def step_static(cfg: RenderConfig, params, cams, images, final_T, targets, n_norm, loss_out, dL, grads,
                counters: Optional[torch.Tensor] = None):
    """One training step through snp_step_static: the workspace is the
    library's static device scratch (no allocation).  `counters` (int64
    device tensor of 8, optional) receives the workspace counters."""
    ccfg = cfg.to_c()
    cams = list(cams)
    pr = L.SnpPrims()
    pr.P = int(params["centers"].shape[0])
    for k in PARAM_KEYS:
        setattr(pr, k, _ptr(params.get(k)))
    g = L.SnpGrads()
    for k, _ in L.SnpGrads._fields_:
        setattr(g, k, _ptr(grads.get(k)))
    cnt = None
    if counters is not None:
        assert counters.is_cuda and counters.dtype == torch.int64 and counters.numel() >= 8
        cnt = C.c_void_p(counters.data_ptr())
    L.check(L.lib().snp_step_static(C.byref(ccfg), C.byref(pr), len(cams), camera_array(cams), _ptr(images),
                                    _ptr(final_T), _ptr(targets), float(n_norm), C.c_void_p(loss_out.data_ptr()),
                                    _ptr(dL), C.byref(g), cnt, _stream()), "snp_step_static")


def kernel_timing(enable: bool):
    L.check(L.lib().snp_kernel_timing(1 if enable else 0), "snp_kernel_timing")


def kernel_timing_read():
    """(forward ms, backward ms) of the last eager rasterizer launches."""
    f, b = C.c_float(), C.c_float()
    L.check(L.lib().snp_kernel_timing_read(C.byref(f), C.byref(b)), "snp_kernel_timing_read")
    return float(f.value), float(b.value)


def zeros_like_params(params: Dict[str, torch.Tensor]) -> Dict[str, torch.Tensor]:
    """Zeroed gradient tensors for the parameters the backward differentiates
    (every one but the Gaussians' opacity)."""
    keys = {k for k, _ in L.SnpGrads._fields_}
    return {k: torch.zeros_like(v) for k, v in params.items() if k in keys}


class GraphStep:
    """A whole training step (zero grads, preprocess, bin, sort, forward, L1
    loss, backward) captured once into a HIP graph and replayed.

    The instance count is only known on the device: a replay whose tile
    instances exceed the workspace capacity, or whose density phases leave
    the supported range, only sets a device flag.  Call check() after
    replays (it synchronises) before trusting their results."""

    def __init__(self, rast: Rasterizer, params, targets: torch.Tensor, n_norm: float):
        self.rast = rast
        self.params = params
        self.images, self.final_T = rast.new_images()
        self.targets = targets
        self.n_norm = float(n_norm)
        self.loss = torch.zeros(1, dtype=torch.float64, device=rast.device)
        self.dL = torch.empty_like(self.images)
        self.grads = zeros_like_params(params)
        self._g = rast.grads_struct(self.grads)
        self._prims = rast._prims(params)
        h = C.c_void_p()
        L.check(L.lib().snp_graph_create(C.byref(rast.ccfg), C.byref(self._prims), rast.V, rast.ccams, rast.ws_ptr,
                                         C.byref(rast.layout), _ptr(self.images), _ptr(self.final_T),
                                         _ptr(self.targets), self.n_norm, C.c_void_p(self.loss.data_ptr()),
                                         _ptr(self.dL), C.byref(self._g), _stream(), C.byref(h)), "snp_graph_create")
        self.handle = h

    def launch(self):
        self.rast.generation += 1
        L.check(L.lib().snp_graph_launch(self.handle, _stream()), "snp_graph_launch")

    def check(self):
        """Synchronises and raises SnpError if a replay overflowed the
        workspace (SNP_ERR_CAPACITY) or met a phase out of range
        (SNP_ERR_RANGE)."""
        self.rast.read_status()

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            L.lib().snp_graph_destroy(h)
            self.handle = None


class ForwardGraph:
    """The forward pipeline alone (preprocess, bin, sort, forward) captured
    once into a HIP graph and replayed: rendering without per-launch host
    overhead (either primitive kind)."""

    def __init__(self, rast: Rasterizer, params, images=None, final_T=None):
        self.rast = rast
        self.params = params
        if images is None:
            images, final_T = rast.new_images()
        self.images, self.final_T = images, final_T
        self._prims = rast._prims(params)
        h = C.c_void_p()
        L.check(L.lib().snp_graph_create_forward(C.byref(rast.ccfg), C.byref(self._prims), rast.V, rast.ccams,
                                                 rast.ws_ptr, C.byref(rast.layout), _ptr(self.images),
                                                 _ptr(self.final_T), _stream(), C.byref(h)),
                "snp_graph_create_forward")
        self.handle = h

    def launch(self):
        self.rast.generation += 1
        L.check(L.lib().snp_graph_launch(self.handle, _stream()), "snp_graph_launch")

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            L.lib().snp_graph_destroy(h)
            self.handle = None


class SplatRender(torch.autograd.Function):
    """images = render(params); backward gives d loss / d params through the
    hand-written adjoint.  Inputs: the Rasterizer, then the parameter tensors
    in PARAM_KEYS order (None for absent ones).

    The backward reads the workspace the forward left (sorted lists, records,
    the pair cache).  If anything has rewritten that workspace since -- a
    second render on the same Rasterizer, a step, a re-allocation -- the
    backward first runs preprocess, bin, sort and forward again from the
    saved parameters (the forward is deterministic, so this restores the
    same workspace and images bit for bit)."""

    @staticmethod
    def forward(ctx, rast: Rasterizer, *tensors):
        params = {k: t for k, t in zip(PARAM_KEYS, tensors) if t is not None}
        params = {k: v.detach().contiguous() for k, v in params.items()}
        rast.prepare(params)
        images, final_T = rast.new_images()
        rast.forward(params, images, final_T)
        ctx.rast = rast
        ctx.generation = rast.generation
        ctx.keys = [k for k, t in zip(PARAM_KEYS, tensors) if t is not None]
        ctx.save_for_backward(images, *[params[k] for k in ctx.keys])
        ctx.mark_non_differentiable(final_T)
        return images, final_T

    @staticmethod
    def backward(ctx, dL_dimages, _dT):
        images, *saved = ctx.saved_tensors
        params = dict(zip(ctx.keys, saved))
        rast = ctx.rast
        if rast.generation != ctx.generation:
            rast.prepare(params)
            again, T = rast.new_images()
            rast.forward(params, again, T)
            images = again
        grads = zeros_like_params(params)
        rast.backward(params, images, dL_dimages.contiguous(), grads)
        out = [None]
        for k in PARAM_KEYS:
            out.append(grads.get(k) if k in params else None)
        return tuple(out)


def splat_render(rast: Rasterizer, params: Dict[str, torch.Tensor]):
    """Differentiable render: returns (images packed per view, final_T)."""
    return SplatRender.apply(rast, *[params.get(k) for k in PARAM_KEYS])
