"""Splattable neural primitives on MI355X: a differentiable tile rasterizer of
ellipsoid-bounded cosine-MLP density primitives, implemented as HIP kernels
for gfx950 behind a C ABI (include/snp.h) with a thin Python binding."""
from .render import (RenderConfig, Rasterizer, GraphStep, ForwardGraph, SplatRender, splat_render, step_static, params_to_device,  # noqa: F401
                     camera_array, zeros_like_params, cmlp_param_count, kernel_timing, kernel_timing_read,
                     PARAM_KEYS)
from ._lib import lib, SnpError  # noqa: F401
