"""Training-step extras on the device, through the C ABI: Adam over all
parameter groups in one launch, the scale regulariser, and population
control by the density-MLP gradient magnitude (Sec. 3.3, "Training" and
"Population Control"; the appendix on hyperparameters).  Argument
marshalling only; every step runs in libsnp's kernels."""
from __future__ import annotations

import ctypes as C
from typing import Dict, Optional

import torch

from . import _lib as L
from .render import Rasterizer, _ptr, _stream

# per-group learning rates of the paper's appendix (MLP 1e-3 covers the
# density and colour networks; constant colours take the SH rate)
PAPER_LRS = {"centers": 1.6e-4, "scales": 5e-3, "quats": 1e-3, "w1": 1e-3, "b1": 1e-3, "w2": 1e-3, "b2": 1e-3,
             "cmlp": 1e-3, "xi": 1e-3, "sh": 2.5e-3, "colors": 2.5e-3}


class Adam:
    """Adam on named device tensors with per-tensor learning rates; `log_space`
    names tensors optimised as log(param) (3DGS's scales)."""

    def __init__(self, params: Dict[str, torch.Tensor], lrs: Optional[Dict[str, float]] = None,
                 log_space=("scales",), betas=(0.9, 0.999), eps=1e-15):
        lrs = PAPER_LRS if lrs is None else lrs
        self.params = params
        self.lrs = {k: float(lrs[k]) for k in params if k in lrs}
        assert len(self.lrs) <= L.MAX_ADAM_GROUPS
        self.log_space = set(log_space)
        self.betas, self.eps = betas, float(eps)
        self.m = {k: torch.zeros_like(params[k]) for k in self.lrs}
        self.v = {k: torch.zeros_like(params[k]) for k in self.lrs}
        self.t = 0

    def step(self, grads: Dict[str, torch.Tensor]):
        self.t += 1
        keys = [k for k in self.lrs if k in grads]
        arr = (L.SnpAdamGroup * max(1, len(keys)))()
        for i, k in enumerate(keys):
            g = arr[i]
            g.param, g.grad = _ptr(self.params[k]), _ptr(grads[k])
            g.m, g.v = _ptr(self.m[k]), _ptr(self.v[k])
            g.n = self.params[k].numel()
            g.lr = self.lrs[k]
            g.log_space = 1 if k in self.log_space else 0
        L.check(L.lib().snp_adam_step(arr, len(keys), self.t, float(self.betas[0]), float(self.betas[1]), self.eps,
                                      _stream()), "snp_adam_step")


def scale_regularizer(rast: Rasterizer, scales: torch.Tensor, weight: float, grad_scales=None, loss_out=None):
    """weight / P * sum_p std(s_p); adds its gradient into grad_scales.
    Returns the loss as a float64 device tensor."""
    loss_out = torch.zeros(1, dtype=torch.float64, device=scales.device) if loss_out is None else loss_out
    L.check(L.lib().snp_scale_regularizer(scales.shape[0], _ptr(scales), float(weight), _ptr(grad_scales),
                                          C.c_void_p(loss_out.data_ptr()), rast.ws_ptr, C.byref(rast.layout),
                                          _stream()), "snp_scale_regularizer")
    return loss_out


def density_control(densify_threshold=1e-4, prune_threshold=2e-6, grow_scale=1e-2, prune_scale=0.5,
                    split_shrink=1.6) -> L.SnpDensityControl:
    dc = L.SnpDensityControl()
    dc.densify_threshold, dc.prune_threshold = densify_threshold, prune_threshold
    dc.grow_scale, dc.prune_scale, dc.split_shrink = grow_scale, prune_scale, split_shrink
    return dc


def densify_accumulate(rast: Rasterizer, grads: Dict[str, torch.Tensor], acc: torch.Tensor, visible: torch.Tensor):
    """acc += ||grad of the density MLP||, visible += covered a tile (the
    rasterizer's last preprocess)."""
    g = rast.grads_struct(grads)
    L.check(L.lib().snp_densify_accumulate(rast.P, rast.cfg.n_hidden, rast.V, C.byref(g), rast.ws_ptr,
                                           C.byref(rast.layout), _ptr(acc), _ptr(visible), _stream()),
            "snp_densify_accumulate")


def densify(params: Dict[str, torch.Tensor], state: Dict[str, torch.Tensor], acc: torch.Tensor,
            visible: torch.Tensor, noise: torch.Tensor, dc: Optional[L.SnpDensityControl] = None):
    """Population control: plan on the device, read the new count (one
    synchronisation), allocate the new tensors and carry every row over.
    params / state: (P, ...) float32 tensors (state: optimizer moments);
    noise: (P, 2, 3) standard normals for split children.
    Returns (new params, new state, action)."""
    dc = density_control() if dc is None else dc
    P = params["centers"].shape[0]
    dev = params["centers"].device
    action = torch.empty(P, dtype=torch.int32, device=dev)
    offsets = torch.empty(P, dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    nbytes = int(L.lib().snp_densify_scratch_bytes(P))
    scratch = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    sp = C.c_void_p(scratch.data_ptr() + (-scratch.data_ptr()) % 256)
    L.check(L.lib().snp_densify_plan(P, _ptr(params["scales"]), _ptr(acc), _ptr(visible), C.byref(dc),
                                     C.c_void_p(action.data_ptr()), C.c_void_p(offsets.data_ptr()),
                                     C.c_void_p(count.data_ptr()), sp, nbytes, _stream()), "snp_densify_plan")
    n_new = int(count.item())
    kinds = {"centers": L.ROWS_CENTERS, "scales": L.ROWS_SCALES}
    new_p = {k: torch.empty((n_new,) + tuple(v.shape[1:]), dtype=v.dtype, device=dev) for k, v in params.items()}
    new_s = {k: torch.empty((n_new,) + tuple(v.shape[1:]), dtype=v.dtype, device=dev) for k, v in state.items()}
    if n_new == 0:  # everything pruned: no rows to carry over
        return new_p, new_s, action
    items = [(params[k], new_p[k], kinds.get(k, L.ROWS_PARAM)) for k in params] + \
            [(state[k], new_s[k], L.ROWS_STATE) for k in state]
    arr = (L.SnpRowArray * len(items))()
    for i, (src, dst, kind) in enumerate(items):
        arr[i].src, arr[i].dst = _ptr(src), _ptr(dst)
        arr[i].width = src[0].numel() if src.shape[0] else 1
        arr[i].kind = kind
    L.check(L.lib().snp_densify_apply(P, C.c_void_p(action.data_ptr()), C.c_void_p(offsets.data_ptr()),
                                      _ptr(params["centers"]), _ptr(params["scales"]), _ptr(params["quats"]),
                                      _ptr(noise), float(dc.split_shrink), arr, len(items), _stream()),
            "snp_densify_apply")
    return new_p, new_s, action
