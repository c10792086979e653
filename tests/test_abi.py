"""CPU-only checks of the C ABI: the library loads, exports every function
include/snp.h declares, and validates arguments on the host (nothing is
enqueued for an invalid call, so no GPU is needed)."""
import ctypes as C
import os
import re

import pytest

import synthetic as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "snp.h")


def _lib():
    from paper_2510_08491_amd import _lib
    return _lib


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(snp_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = _lib().lib()
    names = declared_functions()
    assert "snp_render_forward" in names and "snp_render_backward" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(_lib().EXPORTED)


def _cfg(**kw):
    from paper_2510_08491_amd import RenderConfig
    return RenderConfig(**kw).to_c()


def test_layout_and_validation():
    L = _lib()
    lib = L.lib()
    from paper_2510_08491_amd.render import camera_array
    cams = camera_array(S.make_cameras([(64, 64), (100, 40)], seed=1))
    lay = L.SnpLayout()
    assert lib.snp_workspace_layout(C.byref(_cfg(n_hidden=16)), 1000, 2, cams, 5000, C.byref(lay)) == L.SNP_OK
    assert lay.capacity == 5000 and lay.total_tiles == 16 + 7 * 3 and lay.table_stride == 84
    offs = [lay.counters, lay.loss, lay.cams, lay.table, lay.records, lay.rects, lay.depth_bits, lay.tile_counts,
            lay.offsets, lay.keys, lay.values, lay.ranges, lay.gview, lay.gtable]
    assert all(o % 256 == 0 for o in offs) and max(offs) < lay.bytes
    # the forward's pair cache: one float per (instance, tile pixel), or nothing
    assert lay.ahat_cache_bytes == 4 * 5000 * 256 and lay.ahat_cache % 256 == 0
    assert lay.ahat_cache + lay.ahat_cache_bytes <= lay.bytes
    lay0 = L.SnpLayout()
    assert lib.snp_workspace_layout(C.byref(_cfg(n_hidden=16, fwd_cache=0)), 1000, 2, cams, 5000,
                                    C.byref(lay0)) == L.SNP_OK
    assert lay0.ahat_cache_bytes == 0 and lay0.bytes < lay.bytes
    assert lib.snp_workspace_layout(C.byref(_cfg(fwd_cache=2)), 10, 2, cams, 100, C.byref(lay0)) == L.SNP_ERR_INVALID
    # only the leading instances cached
    c = _cfg(n_hidden=16)
    c.fwd_cache_instances = 1200
    assert lib.snp_workspace_layout(C.byref(c), 1000, 2, cams, 5000, C.byref(lay0)) == L.SNP_OK
    assert lay0.ahat_cache_bytes == 4 * 1200 * 256 and lay0.bytes < lay.bytes
    c.fwd_cache_instances = -1
    assert lib.snp_workspace_layout(C.byref(c), 1000, 2, cams, 5000, C.byref(lay0)) == L.SNP_ERR_INVALID
    # unsupported / invalid configurations are rejected before any device work
    assert lib.snp_workspace_layout(C.byref(_cfg(n_hidden=12)), 10, 2, cams, 100, C.byref(lay)) == L.SNP_ERR_UNSUPPORTED
    assert lib.snp_workspace_layout(C.byref(_cfg(tile_w=12)), 10, 2, cams, 100, C.byref(lay)) == L.SNP_ERR_UNSUPPORTED
    assert lib.snp_workspace_layout(C.byref(_cfg(alpha_max=1.0)), 10, 2, cams, 100, C.byref(lay)) == L.SNP_ERR_INVALID
    assert lib.snp_workspace_layout(C.byref(_cfg(color_mode=5)), 10, 2, cams, 100, C.byref(lay)) == L.SNP_ERR_INVALID
    # the relighting colour needs a supported colour-network shape
    assert lib.snp_workspace_layout(C.byref(_cfg(color_mode=3)), 10, 2, cams, 100,
                                    C.byref(lay)) == L.SNP_ERR_UNSUPPORTED
    assert lib.snp_workspace_layout(C.byref(_cfg(color_mode=3, cmlp_width=16, cmlp_depth=2)), 10, 2, cams, 100,
                                    C.byref(lay)) == L.SNP_OK
    assert lib.snp_workspace_layout(C.byref(_cfg(color_mode=2)), 10, 2, cams, 100, C.byref(lay)) == L.SNP_OK
    assert lib.snp_workspace_layout(C.byref(_cfg()), 0, 2, cams, 100, C.byref(lay)) == L.SNP_ERR_INVALID
    assert lib.snp_workspace_layout(C.byref(_cfg()), 10, 0, cams, 100, C.byref(lay)) == L.SNP_ERR_INVALID
    assert lib.snp_workspace_layout(C.byref(_cfg(color_mode=1, cmlp_width=24, cmlp_depth=2)), 10, 2, cams, 100,
                                    C.byref(lay)) == L.SNP_ERR_UNSUPPORTED
    bad = camera_array(S.make_cameras([(64, 64)], seed=1))
    bad[0].fx = 0.0
    assert lib.snp_workspace_layout(C.byref(_cfg()), 10, 1, bad, 100, C.byref(lay)) == L.SNP_ERR_INVALID
    # a call whose layout does not match its arguments is rejected
    assert lib.snp_workspace_layout(C.byref(_cfg()), 1000, 2, cams, 5000, C.byref(lay)) == L.SNP_OK
    assert lib.snp_bin(C.byref(_cfg()), 999, 2, cams, C.c_void_p(256), C.byref(lay), None) == L.SNP_ERR_INVALID
    assert lib.snp_bin(C.byref(_cfg()), 1000, 2, cams, None, C.byref(lay), None) == L.SNP_ERR_INVALID
    assert lib.snp_status_string(L.SNP_ERR_CAPACITY).decode().startswith("tile instances")


def test_supported_tiles():
    lib = _lib().lib()
    arr = (C.c_int32 * 64)()
    n = lib.snp_supported_tiles(arr, 21)
    triples = [tuple(arr[3 * i:3 * i + 3]) for i in range(n)]
    assert (16, 16, 1) in triples and all(tw * th % (64 * ppl) == 0 for tw, th, ppl in triples)


def test_gaussian_layout_and_forward_only():
    """Gaussian splats (primitive 1): no density table, float64
    discriminants, gradient records or pair cache in the workspace; the
    density-MLP options are not checked; the backward entry points refuse
    before touching any pointer."""
    L = _lib()
    lib = L.lib()
    from paper_2510_08491_amd.render import camera_array
    cams = camera_array(S.make_cameras([(64, 64), (100, 40)], seed=1))
    lay, lay_n = L.SnpLayout(), L.SnpLayout()
    assert lib.snp_workspace_layout(C.byref(_cfg(n_hidden=3, omega0=-1.0, primitive=1)), 1000, 2, cams, 5000,
                                    C.byref(lay)) == L.SNP_OK
    assert lib.snp_workspace_layout(C.byref(_cfg(n_hidden=16)), 1000, 2, cams, 5000, C.byref(lay_n)) == L.SNP_OK
    assert lay.table_stride == 0 and lay.ahat_cache_bytes == 0 and lay.bytes < lay_n.bytes
    assert lay.total_tiles == lay_n.total_tiles and lay.capacity == 5000
    assert lib.snp_workspace_layout(C.byref(_cfg(primitive=2)), 1000, 2, cams, 5000, C.byref(lay)) == L.SNP_ERR_INVALID
    # backward and whole steps are not built for Gaussians
    fake = C.c_void_p(256)
    pr, g = L.SnpPrims(), L.SnpGrads()
    pr.P = 1000
    assert lib.snp_render_backward(C.byref(_cfg(primitive=1)), C.byref(pr), 2, cams, fake, C.byref(lay), fake, fake,
                                   C.byref(g), None) == L.SNP_ERR_UNSUPPORTED
    loss = C.c_double(0)
    assert lib.snp_step(C.byref(_cfg(primitive=1)), C.byref(pr), 2, cams, fake, C.byref(lay), fake, fake, fake, 1.0,
                        C.byref(loss), fake, C.byref(g), None) == L.SNP_ERR_UNSUPPORTED


def test_bin_order_option():
    """bin_order 1 adds the depth-sort buffers of the (view, primitive)
    pairs to the workspace, 2 does not; 0 picks 2 for few pairs (here 2000)
    and 1 for many; others are invalid."""
    L = _lib()
    lib = L.lib()
    from paper_2510_08491_amd.render import camera_array
    cams = camera_array(S.make_cameras([(64, 64), (100, 40)], seed=1))
    lays = {}
    for order in (0, 1, 2):
        lays[order] = L.SnpLayout()
        assert lib.snp_workspace_layout(C.byref(_cfg(n_hidden=8, bin_order=order)), 1000, 2, cams, 5000,
                                        C.byref(lays[order])) == L.SNP_OK
    assert lays[1].bytes > lays[2].bytes == lays[0].bytes
    big = {}
    for order in (0, 1):
        big[order] = L.SnpLayout()
        assert lib.snp_workspace_layout(C.byref(_cfg(n_hidden=8, bin_order=order)), 40000, 2, cams, 5000,
                                        C.byref(big[order])) == L.SNP_OK
    assert big[0].bytes == big[1].bytes
    bad = L.SnpLayout()
    assert lib.snp_workspace_layout(C.byref(_cfg(bin_order=3)), 1000, 2, cams, 5000, C.byref(bad)) == L.SNP_ERR_INVALID


def test_time_must_be_finite():
    L = _lib()
    lib = L.lib()
    from paper_2510_08491_amd.render import camera_array
    cams = camera_array(S.make_cameras([(64, 64)], seed=1))
    lay = L.SnpLayout()
    assert lib.snp_workspace_layout(C.byref(_cfg(time=0.5)), 100, 1, cams, 500, C.byref(lay)) == L.SNP_OK
    assert lib.snp_workspace_layout(C.byref(_cfg(time=float("nan"))), 100, 1, cams, 500,
                                    C.byref(lay)) == L.SNP_ERR_INVALID


def test_training_and_graph_entry_points_validate_on_the_host():
    """Invalid calls of the forward graph and the training extras return
    SNP_ERR_INVALID before anything reaches the device."""
    L = _lib()
    lib = L.lib()
    from paper_2510_08491_amd.render import camera_array
    cams = camera_array(S.make_cameras([(64, 64)], seed=1))
    lay = L.SnpLayout()
    assert lib.snp_workspace_layout(C.byref(_cfg()), 100, 1, cams, 500, C.byref(lay)) == L.SNP_OK
    pr = L.SnpPrims()
    pr.P = 100
    h = C.c_void_p()
    fake = C.c_void_p(256)
    # forward graph: null images / graph handle
    assert lib.snp_graph_create_forward(C.byref(_cfg()), C.byref(pr), 1, cams, fake, C.byref(lay), None, fake, None,
                                        C.byref(h)) == L.SNP_ERR_INVALID
    assert lib.snp_graph_create_forward(C.byref(_cfg()), C.byref(pr), 1, cams, fake, C.byref(lay), fake, fake, None,
                                        None) == L.SNP_ERR_INVALID
    # Adam: step 0, too many groups, beta out of range, a non-empty group without moments
    g = (L.SnpAdamGroup * 1)()
    g[0].n = 0
    assert lib.snp_adam_step(g, 1, 0, 0.9, 0.999, 1e-15, None) == L.SNP_ERR_INVALID
    assert lib.snp_adam_step(g, L.MAX_ADAM_GROUPS + 1, 1, 0.9, 0.999, 1e-15, None) == L.SNP_ERR_INVALID
    assert lib.snp_adam_step(g, 1, 1, 1.0, 0.999, 1e-15, None) == L.SNP_ERR_INVALID
    g[0].n = 10
    g[0].param = g[0].grad = fake
    assert lib.snp_adam_step(g, 1, 1, 0.9, 0.999, 1e-15, None) == L.SNP_ERR_INVALID
    # regulariser: no loss output
    assert lib.snp_scale_regularizer(100, fake, 0.1, None, None, fake, C.byref(lay), None) == L.SNP_ERR_INVALID
    # population control: scratch too small, bad array kind, centres without noise
    dc = L.SnpDensityControl()
    dc.split_shrink = 1.6
    assert lib.snp_densify_plan(100, fake, fake, fake, C.byref(dc), fake, fake, fake, fake, 16,
                                None) == L.SNP_ERR_INVALID
    arr = (L.SnpRowArray * 1)()
    arr[0].src = arr[0].dst = fake
    arr[0].width, arr[0].kind = 3, 7
    assert lib.snp_densify_apply(100, fake, fake, fake, fake, fake, fake, 1.6, arr, 1, None) == L.SNP_ERR_INVALID
    arr[0].kind = L.ROWS_CENTERS
    assert lib.snp_densify_apply(100, fake, fake, fake, fake, fake, None, 1.6, arr, 1, None) == L.SNP_ERR_INVALID
    assert lib.snp_densify_scratch_bytes(100) > 400


def test_tuning_cache_lookup():
    """The autotuner's cache key and lookup: the stored 16-view entry gives
    its tile shape and backward batch; unknown classes give None."""
    from paper_2510_08491_amd import tuning
    cams = S.make_cameras([(640, 480)] * 4 + [(1280, 720)] * 8 + [(1920, 1080)] * 4, seed=1)
    assert tuning.key_of(16, 1, cams) == "gfx950/N16/cm1/V16_MP17"
    assert tuning.lookup(16, 1, cams) == (16, 16, 1, 8)
    assert tuning.lookup(8, 0, S.make_cameras([(64, 64)], seed=1)) is None
    shapes = tuning.supported_shapes()
    assert (16, 16, 1) in shapes and (8, 8, 1) in shapes and len(shapes) == 6


def test_per_ray_colour_configurations():
    """Colour mode 4 is built for N = 8 and 16, width 16 with one hidden
    layer, 16 x 16 tiles with one pixel per thread and backward batches of
    8; other configurations are refused before anything is enqueued, and its
    layout holds the network table, the biases and their gradients."""
    L = _lib()
    lib = L.lib()
    from paper_2510_08491_amd.render import camera_array
    cams = camera_array(S.make_cameras([(64, 64)], seed=3, lights=True))
    ok = dict(n_hidden=16, color_mode=4, cmlp_width=16, cmlp_depth=1)
    lay, lay0 = L.SnpLayout(), L.SnpLayout()
    assert lib.snp_workspace_layout(C.byref(_cfg(**ok)), 1000, 1, cams, 5000, C.byref(lay)) == L.SNP_OK
    assert lib.snp_workspace_layout(C.byref(_cfg(**{**ok, "color_mode": 0})), 1000, 1, cams, 5000,
                                    C.byref(lay0)) == L.SNP_OK
    # table (148 floats), bias (16), their gradients and 12 floats per primitive
    assert lay.bytes - lay0.bytes >= 4 * 1000 * (2 * 148 + 2 * 16 + 12)
    for bad in (dict(cmlp_depth=2), dict(cmlp_width=32), dict(n_hidden=4), dict(n_hidden=32), dict(tile_w=8, tile_h=8),
                dict(px_per_lane=2), dict(bwd_batch=4), dict(primitive=1)):
        c = _cfg(**{**ok, **bad})
        assert lib.snp_workspace_layout(C.byref(c), 1000, 1, cams, 5000, C.byref(lay)) == L.SNP_ERR_UNSUPPORTED, bad
    assert lib.snp_workspace_layout(C.byref(_cfg(**{**ok, "bwd_batch": 8})), 1000, 1, cams, 5000,
                                    C.byref(lay)) == L.SNP_OK
