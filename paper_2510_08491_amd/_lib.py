"""ctypes binding of libsnp.so (include/snp.h): struct mirrors and function
prototypes.  Argument marshalling only; every computation runs in the HIP
library.  Loading fails loudly if the library has not been built."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsnp.so")

SNP_OK, SNP_ERR_INVALID, SNP_ERR_CAPACITY, SNP_ERR_HIP, SNP_ERR_UNSUPPORTED, SNP_ERR_RANGE, SNP_ERR_TOO_LARGE = range(7)


class SnpCamera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("R", C.c_float * 9), ("t", C.c_float * 3),
                ("light", C.c_float * 3)]


class SnpConfig(C.Structure):
    _fields_ = [("n_hidden", C.c_int32), ("omega0", C.c_float), ("color_mode", C.c_int32),
                ("cmlp_width", C.c_int32), ("cmlp_depth", C.c_int32), ("tile_w", C.c_int32),
                ("tile_h", C.c_int32), ("px_per_lane", C.c_int32), ("z_near", C.c_float),
                ("t_eps", C.c_float), ("alpha_min", C.c_float), ("alpha_max", C.c_float),
                ("bg", C.c_float * 3), ("persistent", C.c_int32), ("bwd_batch", C.c_int32),
                ("fwd_cache", C.c_int32), ("fwd_cache_instances", C.c_int64), ("primitive", C.c_int32),
                ("bin_order", C.c_int32), ("time", C.c_float)]


class SnpPrims(C.Structure):
    _fields_ = [("P", C.c_int64)] + [(k, C.c_void_p) for k in
                                     ("centers", "scales", "quats", "w1", "b1", "w2", "b2", "colors", "cmlp", "xi",
                                      "sh", "opacity", "wt", "sh_t")]


class SnpGrads(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in
                ("centers", "scales", "quats", "w1", "b1", "w2", "b2", "colors", "cmlp", "xi", "sh", "wt", "sh_t")]


class SnpLayout(C.Structure):
    _fields_ = [(k, C.c_size_t) for k in
                ("bytes", "cams", "table", "records", "rects", "depth_bits", "tile_counts", "offsets", "keys",
                 "values", "ranges", "counters", "gview", "gtable", "loss", "disc_coef")] + \
               [("capacity", C.c_int64), ("table_stride", C.c_int32), ("total_tiles", C.c_int32),
                ("ahat_cache", C.c_size_t), ("ahat_cache_bytes", C.c_size_t), ("tile_pairs", C.c_size_t)]


class SnpAdamGroup(C.Structure):
    _fields_ = [("param", C.c_void_p), ("grad", C.c_void_p), ("m", C.c_void_p), ("v", C.c_void_p),
                ("n", C.c_int64), ("lr", C.c_float), ("log_space", C.c_int32)]


class SnpDensityControl(C.Structure):
    _fields_ = [(k, C.c_float) for k in
                ("densify_threshold", "prune_threshold", "grow_scale", "prune_scale", "split_shrink")]


class SnpRowArray(C.Structure):
    _fields_ = [("src", C.c_void_p), ("dst", C.c_void_p), ("width", C.c_int32), ("kind", C.c_int32)]


MAX_ADAM_GROUPS = 32
PRUNE, KEEP, CLONE, SPLIT = 0, 1, 2, 3
ROWS_PARAM, ROWS_STATE, ROWS_CENTERS, ROWS_SCALES = 0, 1, 2, 3

_lib = None


def lib():
    """The loaded library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2510_08491_amd.build` "
                           "(there is no fallback path)")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, D, VP = C.POINTER, C.c_int32, C.c_int64, C.c_double, C.c_void_p
    cfg, cams, prims, grads, lay = P(SnpConfig), P(SnpCamera), P(SnpPrims), P(SnpGrads), P(SnpLayout)
    protos = {
        "snp_workspace_layout": [cfg, I64, I32, cams, I64, lay],
        "snp_preprocess": [cfg, prims, I32, cams, VP, lay, VP],
        "snp_bin": [cfg, I64, I32, cams, VP, lay, VP],
        "snp_sort": [cfg, I64, I32, cams, VP, lay, VP],
        "snp_render_forward": [cfg, prims, I32, cams, VP, lay, VP, VP, I32, VP],
        "snp_loss_l1": [cfg, I32, cams, VP, VP, D, VP, lay, VP, VP, VP],
        "snp_render_backward": [cfg, prims, I32, cams, VP, lay, VP, VP, grads, VP],
        "snp_step": [cfg, prims, I32, cams, VP, lay, VP, VP, VP, D, VP, VP, grads, VP],
        "snp_step_static": [cfg, prims, I32, cams, VP, VP, VP, D, VP, VP, grads, VP, VP],
        "snp_graph_create": [cfg, prims, I32, cams, VP, lay, VP, VP, VP, D, VP, VP, grads, VP, P(VP)],
        "snp_graph_create_forward": [cfg, prims, I32, cams, VP, lay, VP, VP, VP, P(VP)],
        "snp_graph_launch": [VP, VP],
        "snp_graph_destroy": [VP],
        "snp_read_status": [VP, lay, P(I64), P(I64), VP],
        "snp_supported_tiles": [P(I32), I32],
        "snp_selftest_wave_sum": [VP, VP, I32, VP],
        "snp_read_counters": [VP, lay, P(I64), VP],
        "snp_kernel_timing": [I32],
        "snp_kernel_timing_read": [P(C.c_float), P(C.c_float)],
        "snp_adam_step": [P(SnpAdamGroup), I32, I64, D, D, D, VP],
        "snp_scale_regularizer": [I64, VP, C.c_float, VP, VP, VP, lay, VP],
        "snp_densify_accumulate": [I64, I32, I32, grads, VP, lay, VP, VP, VP],
        "snp_densify_plan": [I64, VP, VP, VP, P(SnpDensityControl), VP, VP, VP, VP, C.c_size_t, VP],
        "snp_densify_apply": [I64, VP, VP, VP, VP, VP, VP, C.c_float, P(SnpRowArray), I32, VP],
    }
    for name, args in protos.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int32
    L.snp_status_string.argtypes = [C.c_int32]
    L.snp_status_string.restype = C.c_char_p
    L.snp_densify_scratch_bytes.argtypes = [I64]
    L.snp_densify_scratch_bytes.restype = C.c_size_t
    _lib = L
    return L


EXPORTED = ["snp_workspace_layout", "snp_preprocess", "snp_bin", "snp_sort", "snp_render_forward", "snp_loss_l1",
            "snp_render_backward", "snp_step", "snp_step_static", "snp_graph_create", "snp_graph_create_forward", "snp_graph_launch",
            "snp_graph_destroy",
            "snp_read_status", "snp_supported_tiles", "snp_status_string", "snp_selftest_wave_sum",
            "snp_read_counters", "snp_kernel_timing", "snp_kernel_timing_read", "snp_adam_step",
            "snp_scale_regularizer", "snp_densify_accumulate", "snp_densify_scratch_bytes", "snp_densify_plan",
            "snp_densify_apply"]


class SnpError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = lib().snp_status_string(code).decode()
        super().__init__(f"{where}: {msg} (status {code})")


def check(code, where):
    if code != SNP_OK:
        raise SnpError(code, where)
