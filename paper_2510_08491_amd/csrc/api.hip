// C ABI of libsnp: argument validation, workspace layout and the sequence of
// kernel launches of each stage.  No entry point allocates device memory;
// everything lives in the caller's workspace.
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "snp_internal.h"

namespace snp {

static inline size_t align256(size_t x) { return (x + 255) / 256 * 256; }

struct Plan {
  snp_layout L;
  size_t scan_scratch, sort_scratch, loss_partials, cams_bytes;
  size_t keys_alt, values_alt;
  size_t dkeys[2], dvals[2], counts_sorted;  // depth sort of the (view, primitive) pairs
  size_t tkeys[2], tvals[2], tile_n;          // persistent launches: tile order by instance count
  std::vector<int32_t> tile_base;
  std::vector<int64_t> pix_base;
  int64_t total_pixels;
  int tile_bits;  // significant bits of the global tile id
  bool depth_first;  // depth sort of the pairs, then the instances by tile bits only
  bool tile_order_on;  // persistent launches take the tiles by instance count, descending
  // colour mode 4: the colour network's table and biases, their gradients,
  // and the rotation / scale gradients handed to the preprocess adjoint
  size_t ctab, cbias, gctab, gcbias, extra_rs;
};

static bool valid_n(int n) { return n == 4 || n == 8 || n == 16 || n == 32; }

static bool gaussian(const snp_config* cfg) { return cfg->primitive == 1; }

static snp_status check_cfg(const snp_config* cfg) {
  if (!cfg) return SNP_ERR_INVALID;
  if (cfg->primitive != 0 && cfg->primitive != 1) return SNP_ERR_INVALID;
  if (!gaussian(cfg)) {
    if (!valid_n(cfg->n_hidden)) return SNP_ERR_UNSUPPORTED;
    if (!(cfg->omega0 > 0.f) || !std::isfinite(cfg->omega0)) return SNP_ERR_INVALID;
  }
  if (cfg->color_mode < 0 || cfg->color_mode > 4) return SNP_ERR_INVALID;
  if ((cfg->color_mode == 1 || cfg->color_mode == 3) && !cmlp_supported(cfg->cmlp_width, cfg->cmlp_depth))
    return SNP_ERR_UNSUPPORTED;
  if (cfg->color_mode == 4 &&
      (gaussian(cfg) || !ray_colour_supported(cfg->cmlp_width, cfg->cmlp_depth) ||
       !ray_colour_raster_supported(cfg->n_hidden, cfg->tile_w, cfg->tile_h, cfg->px_per_lane, cfg->bwd_batch)))
    return SNP_ERR_UNSUPPORTED;
  if (!tile_supported(cfg->tile_w, cfg->tile_h, cfg->px_per_lane)) return SNP_ERR_UNSUPPORTED;
  if (!(cfg->z_near > 0.f)) return SNP_ERR_INVALID;
  if (!(cfg->t_eps >= 0.f && cfg->t_eps < 1.f)) return SNP_ERR_INVALID;
  if (!(cfg->alpha_min >= 0.f && cfg->alpha_max > 0.f && cfg->alpha_max < 1.f)) return SNP_ERR_INVALID;
  if (cfg->persistent != 0 && cfg->persistent != 1) return SNP_ERR_INVALID;
  if (cfg->bwd_batch != 0 && !bwd_batch_supported(cfg->tile_w, cfg->tile_h, cfg->bwd_batch))
    return SNP_ERR_UNSUPPORTED;
  if (cfg->fwd_cache != 0 && cfg->fwd_cache != 1) return SNP_ERR_INVALID;
  if (cfg->fwd_cache_instances < 0) return SNP_ERR_INVALID;
  if (cfg->bin_order < 0 || cfg->bin_order > 2) return SNP_ERR_INVALID;
  if (!std::isfinite(cfg->time)) return SNP_ERR_INVALID;
  return SNP_OK;
}

static snp_status check_cams(int32_t V, const snp_camera* cams) {
  if (V <= 0 || V > 4096 || !cams) return SNP_ERR_INVALID;
  for (int v = 0; v < V; ++v) {
    const snp_camera& c = cams[v];
    if (c.width <= 0 || c.height <= 0 || c.width > 16384 || c.height > 16384) return SNP_ERR_INVALID;
    if (!(c.fx > 0.f) || !(c.fy > 0.f)) return SNP_ERR_INVALID;
    for (int k = 0; k < 9; ++k)
      if (!std::isfinite(c.R[k])) return SNP_ERR_INVALID;
    const double det = (double)c.R[0] * ((double)c.R[4] * c.R[8] - (double)c.R[5] * c.R[7]) -
                       (double)c.R[1] * ((double)c.R[3] * c.R[8] - (double)c.R[5] * c.R[6]) +
                       (double)c.R[2] * ((double)c.R[3] * c.R[7] - (double)c.R[4] * c.R[6]);
    if (!(std::fabs(det) > 1e-6)) return SNP_ERR_INVALID;
  }
  return SNP_OK;
}

static snp_status make_plan(const snp_config* cfg, int64_t P, int32_t V, const snp_camera* cams, int64_t cap,
                            Plan* pl) {
  snp_status s = check_cfg(cfg);
  if (s != SNP_OK) return s;
  s = check_cams(V, cams);
  if (s != SNP_OK) return s;
  if (P <= 0 || P > ((int64_t)1 << 31) - 1) return SNP_ERR_INVALID;
  if ((int64_t)V * P >= ((int64_t)1 << 32)) return SNP_ERR_INVALID;  // pair indices are uint32
  if (cap <= 0 || cap > ((int64_t)1 << 31) - 1) return SNP_ERR_INVALID;
  pl->tile_base.resize(V);
  pl->pix_base.resize(V);
  int64_t tiles = 0, pix = 0;
  for (int v = 0; v < V; ++v) {
    pl->tile_base[v] = (int32_t)tiles;
    pl->pix_base[v] = pix;
    tiles += (int64_t)((cams[v].width + cfg->tile_w - 1) / cfg->tile_w) * ((cams[v].height + cfg->tile_h - 1) / cfg->tile_h);
    pix += (int64_t)cams[v].width * cams[v].height;
  }
  if (tiles >= ((int64_t)1 << 30)) return SNP_ERR_INVALID;
  pl->total_pixels = pix;
  int tb = 1;
  while (((int64_t)1 << tb) < tiles) ++tb;
  pl->tile_bits = tb;
  // the heaviest-first order pays for its sort where tiles are expensive (neural
  // primitives); the Gaussians' cheap tiles do not need it
  pl->tile_order_on = cfg->persistent != 0 && cfg->primitive == 0;
  pl->depth_first = cfg->bin_order == 1 || (cfg->bin_order == 0 && (int64_t)V * P >= ((int64_t)1 << 16));
  // Gaussians have no density table, float64 discriminants, backward arrays
  // or pair cache
  const bool gs = gaussian(cfg);
  const int TS = gs ? 0 : table_stride(cfg->n_hidden);
  const int64_t VP = (int64_t)V * P;
  snp_layout& L = pl->L;
  std::memset(&L, 0, sizeof(L));
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  L.counters = take(sizeof(unsigned long long) * CNT_COUNT);
  L.loss = take(loss_scratch_bytes());
  pl->loss_partials = L.loss;
  L.cams = take(sizeof(CamDev) * (size_t)V);
  L.table = take(sizeof(float) * (size_t)P * TS);
  L.records = take(sizeof(float) * (size_t)VP * kRecFloats);
  L.disc_coef = take(gs ? 0 : sizeof(double) * 6 * (size_t)VP);
  L.rects = take(sizeof(int32_t) * 4 * (size_t)VP);
  L.depth_bits = take(sizeof(uint32_t) * (size_t)VP);
  L.tile_counts = take(sizeof(uint32_t) * (size_t)VP);
  L.offsets = take(sizeof(uint32_t) * (size_t)VP);
  pl->scan_scratch = take(scan_scratch_bytes(VP));
  const size_t dn = pl->depth_first ? (size_t)VP : 0;
  for (int k = 0; k < 2; ++k) {
    pl->dkeys[k] = take(sizeof(unsigned long long) * dn);
    pl->dvals[k] = take(sizeof(uint32_t) * dn);
  }
  pl->counts_sorted = take(sizeof(uint32_t) * dn);
  L.keys = take(sizeof(unsigned long long) * (size_t)cap);
  pl->keys_alt = take(sizeof(unsigned long long) * (size_t)cap);
  L.values = take(sizeof(uint32_t) * (size_t)cap);
  pl->values_alt = take(sizeof(uint32_t) * (size_t)cap);
  int64_t sort_n = pl->depth_first && VP > cap ? VP : cap;
  if (pl->tile_order_on && tiles > sort_n) sort_n = tiles;
  pl->sort_scratch = take(sort_scratch_bytes(sort_n));
  L.ranges = take(sizeof(uint32_t) * 2 * (size_t)tiles);
  L.tile_pairs = take(sizeof(uint32_t) * (size_t)tiles);
  const size_t tn = pl->tile_order_on ? (size_t)tiles : 0;
  for (int k = 0; k < 2; ++k) {
    pl->tkeys[k] = take(sizeof(unsigned long long) * tn);
    pl->tvals[k] = take(sizeof(uint32_t) * tn);
  }
  pl->tile_n = take(sizeof(unsigned long long));
  L.gview = take(gs ? 0 : sizeof(float) * (size_t)VP * kGViewFloats);
  L.gtable = take(sizeof(float) * (size_t)P * TS);
  {
    const bool rc = cfg->color_mode == 4 && !gs;
    const size_t cts = rc ? (size_t)ray_colour_stride(cfg->cmlp_width, cfg->cmlp_depth) : 0;
    const size_t cw = rc ? (size_t)cfg->cmlp_width : 0;
    pl->ctab = take(sizeof(float) * (size_t)P * cts);
    pl->cbias = take(sizeof(float) * (size_t)VP * cw);
    pl->gctab = take(sizeof(float) * (size_t)P * cts);
    pl->gcbias = take(sizeof(float) * (size_t)VP * cw);
    pl->extra_rs = take(rc ? sizeof(float) * 12 * (size_t)P : 0);
  }
  if (cfg->fwd_cache && !gs) {
    const int64_t n = cfg->fwd_cache_instances > 0 && cfg->fwd_cache_instances < cap ? cfg->fwd_cache_instances : cap;
    L.ahat_cache_bytes = sizeof(float) * (size_t)n * (size_t)(cfg->tile_w * cfg->tile_h);
    L.ahat_cache = take(L.ahat_cache_bytes);
  }
  L.bytes = off;
  L.capacity = cap;
  L.table_stride = TS;
  L.total_tiles = (int32_t)tiles;
  return SNP_OK;
}

static snp_status check_ws(const Plan& pl, void* ws, size_t ws_bytes) {
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0) return SNP_ERR_INVALID;
  if (ws_bytes < pl.L.bytes) return SNP_ERR_INVALID;
  return SNP_OK;
}

static snp_status check_prims(const snp_config* cfg, const snp_prims* pr) {
  if (!pr || pr->P <= 0) return SNP_ERR_INVALID;
  if (!pr->centers || !pr->scales || !pr->quats) return SNP_ERR_INVALID;
  if (gaussian(cfg) ? !pr->opacity : (!pr->w1 || !pr->b1 || !pr->w2 || !pr->b2)) return SNP_ERR_INVALID;
  if (cfg->color_mode == 0 && !pr->colors) return SNP_ERR_INVALID;
  if (cfg->color_mode == 1 && (!pr->cmlp || !pr->xi)) return SNP_ERR_INVALID;
  if (cfg->color_mode == 2 && !pr->sh) return SNP_ERR_INVALID;
  if (cfg->color_mode == 3 && (!pr->cmlp || !pr->xi || !pr->colors)) return SNP_ERR_INVALID;
  if (cfg->color_mode == 4 && (!pr->cmlp || !pr->colors)) return SNP_ERR_INVALID;
  return SNP_OK;
}

#define SNP_HIP(x)                          \
  do {                                      \
    if ((x) != hipSuccess) return SNP_ERR_HIP; \
  } while (0)

template <typename T>
static T* wsp(void* ws, size_t off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(ws) + off);
}

// the time-dependent zero-order SH term: the coefficient array and the 12
// functions of xi_t (xi^1..4, cos(i xi), sin(i xi)) it multiplies
static void sh_time(const snp_config* cfg, const snp_prims* pr, ShArgs* sa) {
  sa->sh_t = pr->sh_t;
  const double t = cfg->time;
  for (int i = 1; i <= 4; ++i) {
    sa->tb[i - 1] = (float)std::pow(t, i);
    sa->tb[3 + i] = (float)std::cos(i * t);
    sa->tb[7 + i] = (float)std::sin(i * t);
  }
}

static RayColourArgs ray_colour_args(const snp_config* cfg, const snp_prims* pr, int32_t V, const Plan& pl,
                                     void* ws) {
  RayColourArgs ra;
  std::memset(&ra, 0, sizeof(ra));
  ra.P = pr->P;
  ra.V = V;
  ra.W = cfg->cmlp_width;
  ra.D = cfg->cmlp_depth;
  ra.centers = pr->centers;
  ra.scales = pr->scales;
  ra.quats = pr->quats;
  ra.cmlp = pr->cmlp;
  ra.cams = wsp<CamDev>(ws, pl.L.cams);
  ra.tile_counts = wsp<uint32_t>(ws, pl.L.tile_counts);
  ra.ctab = wsp<float>(ws, pl.ctab);
  ra.cbias = wsp<float>(ws, pl.cbias);
  ra.gctab = wsp<float>(ws, pl.gctab);
  ra.gcbias = wsp<float>(ws, pl.gcbias);
  ra.extra_rs = wsp<float>(ws, pl.extra_rs);
  return ra;
}

static snp_status do_preprocess(const snp_config* cfg, const snp_prims* pr, int32_t V, const snp_camera* cams,
                                const Plan& pl, void* ws, hipStream_t st) {
  const snp_layout& L = pl.L;
  unsigned long long* counters = wsp<unsigned long long>(ws, L.counters);
  CamDev* cd = wsp<CamDev>(ws, L.cams);
  SNP_HIP(zero_counters(counters, CNT_COUNT, st));
  for (int v0 = 0; v0 < V; v0 += kMaxCamsPerChunk) {
    CamChunk ch;
    std::memset(&ch, 0, sizeof(ch));
    ch.first = v0;
    ch.count = std::min(kMaxCamsPerChunk, V - v0);
    ch.tile_w = cfg->tile_w;
    ch.tile_h = cfg->tile_h;
    for (int i = 0; i < ch.count; ++i) {
      ch.cam[i] = cams[v0 + i];
      ch.tile_base[i] = pl.tile_base[v0 + i];
      ch.pix_base[i] = pl.pix_base[v0 + i];
    }
    SNP_HIP(launch_setup_cams(ch, cd, st));
  }
  if (!gaussian(cfg))
    SNP_HIP(launch_prim_table(cfg->n_hidden, pr->P, cfg->omega0, cfg->time, *pr, wsp<float>(ws, L.table), counters,
                              st));
  ViewArgs va;
  va.P = pr->P;
  va.V = V;
  va.z_near = cfg->z_near;
  va.color_mode = cfg->color_mode;
  va.primitive = cfg->primitive;
  va.opacity = pr->opacity;
  va.centers = pr->centers;
  va.scales = pr->scales;
  va.quats = pr->quats;
  va.colors = pr->colors;
  va.cams = cd;
  va.records = wsp<float>(ws, L.records);
  va.rects = wsp<int32_t>(ws, L.rects);
  va.depth_bits = wsp<uint32_t>(ws, L.depth_bits);
  va.tile_counts = wsp<uint32_t>(ws, L.tile_counts);
  va.disc_coef = wsp<double>(ws, L.disc_coef);
  SNP_HIP(launch_preprocess_views(va, st));
  if (cfg->color_mode == 1 || cfg->color_mode == 3) {
    CmlpArgs ca;
    std::memset(&ca, 0, sizeof(ca));
    ca.P = pr->P;
    ca.V = V;
    ca.relight = cfg->color_mode == 3;
    ca.centers = pr->centers;
    ca.xi = pr->xi;
    ca.cmlp = pr->cmlp;
    ca.colors = pr->colors;
    ca.cams = cd;
    ca.tile_counts = va.tile_counts;
    ca.records = va.records;
    SNP_HIP(launch_cmlp_fwd(cfg->cmlp_width, cfg->cmlp_depth, ca, st));
  }
  if (cfg->color_mode == 2) {
    ShArgs sa;
    std::memset(&sa, 0, sizeof(sa));
    sa.P = pr->P;
    sa.V = V;
    sa.centers = pr->centers;
    sa.sh = pr->sh;
    sh_time(cfg, pr, &sa);
    sa.cams = cd;
    sa.tile_counts = va.tile_counts;
    sa.records = va.records;
    SNP_HIP(launch_sh_fwd(sa, st));
  }
  if (cfg->color_mode == 4) SNP_HIP(launch_ray_colour_fwd(ray_colour_args(cfg, pr, V, pl, ws), st));
  return SNP_OK;
}

constexpr int kDepthBits = 31;  // positive float32 depth: the sign bit is zero
constexpr int kTileKeyBits = 16;  // instance count of a tile, saturated, for the work-queue order

// key bits the instance sort orders: the tile bits only when the instances
// are emitted in depth order, else depth and tile bits
static int sort_lo(const Plan& pl) { return pl.depth_first ? kDepthBits : 0; }
static int sort_bits(const Plan& pl) { return pl.depth_first ? pl.tile_bits : kDepthBits + pl.tile_bits; }

// Instance offsets and instances, in primitive order or (depth_first) in the
// depth order of the (view, primitive) pairs.
static snp_status do_bin(const snp_config* cfg, int64_t P, int32_t V, const Plan& pl, void* ws, hipStream_t st) {
  const snp_layout& L = pl.L;
  unsigned long long* counters = wsp<unsigned long long>(ws, L.counters);
  const int64_t VP = (int64_t)V * P;
  const uint32_t* order = nullptr;  // identity: primitive order
  const uint32_t* counts = wsp<uint32_t>(ws, L.tile_counts);
  if (pl.depth_first) {
    unsigned long long* dk0 = wsp<unsigned long long>(ws, pl.dkeys[0]);
    unsigned long long* dk1 = wsp<unsigned long long>(ws, pl.dkeys[1]);
    uint32_t* dv0 = wsp<uint32_t>(ws, pl.dvals[0]);
    uint32_t* dv1 = wsp<uint32_t>(ws, pl.dvals[1]);
    SNP_HIP(launch_depth_keys(wsp<uint32_t>(ws, L.depth_bits), VP, dk0, dv0, counters + CNT_DEPTH_SORT, st));
    SNP_HIP(radix_sort(dk0, dv0, dk1, dv1, VP, counters + CNT_DEPTH_SORT, 0, kDepthBits,
                       wsp<void>(ws, pl.sort_scratch), st));
    order = radix_passes(kDepthBits) % 2 == 1 ? dv1 : dv0;
    uint32_t* cs = wsp<uint32_t>(ws, pl.counts_sorted);
    SNP_HIP(launch_gather_counts(order, counts, VP, cs, st));
    counts = cs;
  }
  SNP_HIP(scan_exclusive_u32(counts, wsp<uint32_t>(ws, L.offsets), VP, wsp<void>(ws, pl.scan_scratch),
                             reinterpret_cast<uint64_t*>(counters + CNT_INSTANCES), st));
  const bool odd = radix_passes(sort_bits(pl)) % 2 == 1;
  EmitArgs ea;
  ea.P = P;
  ea.V = V;
  ea.capacity = L.capacity;
  ea.cams = wsp<CamDev>(ws, L.cams);
  ea.rects = wsp<int32_t>(ws, L.rects);
  ea.depth_bits = wsp<uint32_t>(ws, L.depth_bits);
  ea.tile_counts = wsp<uint32_t>(ws, L.tile_counts);
  ea.order = order;
  ea.offsets = wsp<uint32_t>(ws, L.offsets);
  ea.keys = wsp<unsigned long long>(ws, odd ? pl.keys_alt : L.keys);
  ea.values = wsp<uint32_t>(ws, odd ? pl.values_alt : L.values);
  SNP_HIP(launch_emit(ea, counters, st));
  (void)cfg;
  return SNP_OK;
}

static snp_status do_sort(const Plan& pl, void* ws, hipStream_t st) {
  const snp_layout& L = pl.L;
  unsigned long long* counters = wsp<unsigned long long>(ws, L.counters);
  const bool odd = radix_passes(sort_bits(pl)) % 2 == 1;
  unsigned long long* k_main = wsp<unsigned long long>(ws, L.keys);
  unsigned long long* k_alt = wsp<unsigned long long>(ws, pl.keys_alt);
  uint32_t* v_main = wsp<uint32_t>(ws, L.values);
  uint32_t* v_alt = wsp<uint32_t>(ws, pl.values_alt);
  // instances emitted in depth order need their tile bits sorted only: the
  // passes are stable, which completes the (tile, depth) order
  unsigned long long* n_inst = counters + CNT_INSTANCES;
  void* scr = wsp<void>(ws, pl.sort_scratch);
  if (odd)
    SNP_HIP(radix_sort(k_alt, v_alt, k_main, v_main, L.capacity, n_inst, sort_lo(pl), sort_bits(pl), scr, st));
  else
    SNP_HIP(radix_sort(k_main, v_main, k_alt, v_alt, L.capacity, n_inst, sort_lo(pl), sort_bits(pl), scr, st));
  SNP_HIP(launch_ranges(k_main, counters, L.capacity, wsp<uint32_t>(ws, L.ranges), L.total_tiles, st));
  if (pl.tile_order_on) {
    // tiles by instance count, descending, for the persistent rasterizers' work queue
    unsigned long long* tk0 = wsp<unsigned long long>(ws, pl.tkeys[0]);
    unsigned long long* tk1 = wsp<unsigned long long>(ws, pl.tkeys[1]);
    uint32_t* tv0 = wsp<uint32_t>(ws, pl.tvals[0]);
    uint32_t* tv1 = wsp<uint32_t>(ws, pl.tvals[1]);
    unsigned long long* tn = wsp<unsigned long long>(ws, pl.tile_n);
    SNP_HIP(launch_tile_keys(wsp<uint32_t>(ws, L.ranges), L.total_tiles, tk0, tv0, tn, st));
    SNP_HIP(radix_sort(tk0, tv0, tk1, tv1, L.total_tiles, tn, 0, kTileKeyBits, wsp<void>(ws, pl.sort_scratch), st));
  }
  return SNP_OK;
}

static int64_t L_tiles(const Plan& pl) { return pl.L.total_tiles; }

static RasterArgs raster_args(const snp_config* cfg, int64_t P, int32_t V, const Plan& pl, void* ws) {
  const snp_layout& L = pl.L;
  RasterArgs a;
  std::memset(&a, 0, sizeof(a));
  a.cams = wsp<CamDev>(ws, L.cams);
  a.V = V;
  a.P = P;
  a.total_tiles = L.total_tiles;
  a.table = wsp<float>(ws, L.table);
  a.records = wsp<float>(ws, L.records);
  a.values = wsp<uint32_t>(ws, L.values);
  a.ranges = wsp<uint32_t>(ws, L.ranges);
  // the sorted tile ids (2 passes over the 16 key bits: back in the first buffer)
  a.tile_order = pl.tile_order_on ? wsp<uint32_t>(ws, pl.tvals[radix_passes(kTileKeyBits) % 2]) : nullptr;
  a.rects = wsp<int32_t>(ws, L.rects);
  a.gview = wsp<float>(ws, L.gview);
  a.gtable = wsp<float>(ws, L.gtable);
  a.disc_coef = wsp<double>(ws, L.disc_coef);
  a.ahat_cache = cfg->fwd_cache ? wsp<float>(ws, L.ahat_cache) : nullptr;
  a.cache_instances = cfg->fwd_cache ? (int64_t)(L.ahat_cache_bytes / (sizeof(float) * cfg->tile_w * cfg->tile_h)) : 0;
  a.counters = wsp<unsigned long long>(ws, L.counters);
  a.tile_pairs = wsp<uint32_t>(ws, L.tile_pairs);
  if (cfg->color_mode == 4) {
    a.ctab = wsp<float>(ws, pl.ctab);
    a.cbias = wsp<float>(ws, pl.cbias);
    a.gctab = wsp<float>(ws, pl.gctab);
    a.gcbias = wsp<float>(ws, pl.gcbias);
  }
  a.t_eps = cfg->t_eps;
  a.alpha_min = cfg->alpha_min;
  a.alpha_max = cfg->alpha_max;
  a.bg0 = cfg->bg[0];
  a.bg1 = cfg->bg[1];
  a.bg2 = cfg->bg[2];
  return a;
}

// Optional events around the rasterizer launches (eager calls only), for
// measuring the kernels' own durations.
struct KernelTimer {
  bool on = false, have_fwd = false, have_bwd = false;
  hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
};
static KernelTimer g_timer;

static bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) return true;
  return cs != hipStreamCaptureStatusNone;
}

static void timer_mark(int which, hipStream_t st) {
  if (!g_timer.on || capturing(st)) return;
  (void)hipEventRecord(g_timer.e[which], st);
  if (which == 1) g_timer.have_fwd = true;
  if (which == 3) g_timer.have_bwd = true;
}

// depth of the per-ray colour network the rasterizers evaluate (0: none)
static int ray_depth(const snp_config* cfg) { return cfg->color_mode == 4 ? cfg->cmlp_depth : 0; }

static snp_status do_forward(const snp_config* cfg, int64_t P, int32_t V, const Plan& pl, void* ws, float* images,
                             float* final_T, int count, hipStream_t st) {
  RasterArgs a = raster_args(cfg, P, V, pl, ws);
  a.images = images;
  a.final_T = final_T;
  if (cfg->persistent) SNP_HIP(zero_counter(a.counters + CNT_QUEUE_FWD, st));
  if (count) SNP_HIP(fill_u32(a.tile_pairs, L_tiles(pl), 0u, st));
  timer_mark(0, st);
  if (gaussian(cfg))
    SNP_HIP(launch_render_fwd_gauss(cfg->tile_w, cfg->tile_h, cfg->px_per_lane, cfg->persistent != 0, count != 0, a,
                                    st));
  else
    SNP_HIP(launch_render_fwd(cfg->n_hidden, cfg->tile_w, cfg->tile_h, cfg->px_per_lane, cfg->persistent != 0,
                              count != 0, ray_depth(cfg), a, st));
  timer_mark(1, st);
  return SNP_OK;
}

static snp_status do_backward(const snp_config* cfg, const snp_prims* pr, int32_t V, const Plan& pl, void* ws,
                              const float* images, const float* dL, const snp_grads* g, hipStream_t st) {
  const snp_layout& L = pl.L;
  const int64_t P = pr->P;
  RasterArgs a = raster_args(cfg, P, V, pl, ws);
  a.images_in = images;
  a.dL = dL;
  SNP_HIP(zero_f32(a.gview, (int64_t)V * P * kGViewFloats, st));
  SNP_HIP(zero_f32(a.gtable, P * (int64_t)L.table_stride, st));
  if (cfg->persistent) SNP_HIP(zero_counter(a.counters + CNT_QUEUE_BWD, st));
  if (cfg->color_mode == 4) {
    SNP_HIP(zero_f32(a.gctab, P * (int64_t)ray_colour_stride(cfg->cmlp_width, cfg->cmlp_depth), st));
    SNP_HIP(zero_f32(a.gcbias, (int64_t)V * P * cfg->cmlp_width, st));
  }
  timer_mark(2, st);
  const int nb = cfg->bwd_batch ? cfg->bwd_batch : bwd_batch_default(cfg->tile_w, cfg->tile_h);
  SNP_HIP(launch_render_bwd(cfg->n_hidden, cfg->tile_w, cfg->tile_h, nb, cfg->persistent != 0, ray_depth(cfg), a,
                            st));
  timer_mark(3, st);
  if (cfg->color_mode == 4) {
    RayColourArgs ra = ray_colour_args(cfg, pr, V, pl, ws);
    ra.g_cmlp = g->cmlp;
    ra.g_centers = g->centers;
    SNP_HIP(launch_ray_colour_bwd(ra, st));
  }
  if (cfg->color_mode == 1 || cfg->color_mode == 3) {
    CmlpArgs ca;
    std::memset(&ca, 0, sizeof(ca));
    ca.P = P;
    ca.V = V;
    ca.relight = cfg->color_mode == 3;
    ca.centers = pr->centers;
    ca.xi = pr->xi;
    ca.cmlp = pr->cmlp;
    ca.colors = pr->colors;
    ca.g_centers = cfg->color_mode == 3 ? g->centers : nullptr;
    ca.cams = a.cams;
    ca.tile_counts = wsp<uint32_t>(ws, L.tile_counts);
    ca.records = wsp<float>(ws, L.records);
    ca.gview = a.gview;
    ca.g_cmlp = g->cmlp;
    ca.g_xi = g->xi;
    // also without g->cmlp: the view-direction gradient feeds the centres
    if (g->cmlp || g->xi || g->centers) SNP_HIP(launch_cmlp_bwd(cfg->cmlp_width, cfg->cmlp_depth, ca, st));
  }
  if (cfg->color_mode == 2 && (g->sh || g->centers || g->sh_t)) {
    // also without g->sh: the view-direction gradient feeds the centres
    ShArgs sa;
    std::memset(&sa, 0, sizeof(sa));
    sa.P = P;
    sa.V = V;
    sa.centers = pr->centers;
    sa.sh = pr->sh;
    sh_time(cfg, pr, &sa);
    sa.g_sh_t = g->sh_t;
    sa.cams = a.cams;
    sa.tile_counts = wsp<uint32_t>(ws, L.tile_counts);
    sa.records = wsp<float>(ws, L.records);
    sa.gview = a.gview;
    sa.g_sh = g->sh;
    SNP_HIP(launch_sh_bwd(sa, st));
  }
  PreBwdArgs pa;
  pa.P = P;
  pa.V = V;
  pa.N = cfg->n_hidden;
  pa.color_mode = cfg->color_mode;
  pa.omega0 = cfg->omega0;
  pa.time = pr->wt ? cfg->time : 0.f;
  pa.centers = pr->centers;
  pa.scales = pr->scales;
  pa.quats = pr->quats;
  pa.w1 = pr->w1;
  pa.cams = a.cams;
  pa.records = wsp<float>(ws, L.records);
  pa.tile_counts = wsp<uint32_t>(ws, L.tile_counts);
  pa.gview = a.gview;
  pa.gtable = a.gtable;
  pa.extra_rs = cfg->color_mode == 4 ? wsp<float>(ws, pl.extra_rs) : nullptr;
  pa.g = *g;
  SNP_HIP(launch_preprocess_bwd(pa, st));
  return SNP_OK;
}

static snp_status zero_grads(const snp_config* cfg, int64_t P, const snp_grads* g, hipStream_t st) {
  const int64_t N = cfg->n_hidden;
  SNP_HIP(zero_f32(g->centers, 3 * P, st));
  SNP_HIP(zero_f32(g->scales, 3 * P, st));
  SNP_HIP(zero_f32(g->quats, 4 * P, st));
  SNP_HIP(zero_f32(g->w1, 3 * N * P, st));
  SNP_HIP(zero_f32(g->b1, N * P, st));
  SNP_HIP(zero_f32(g->w2, N * P, st));
  SNP_HIP(zero_f32(g->b2, P, st));
  if (cfg->color_mode == 0 || cfg->color_mode == 3 || cfg->color_mode == 4) SNP_HIP(zero_f32(g->colors, 3 * P, st));
  if (cfg->color_mode == 4)
    SNP_HIP(zero_f32(g->cmlp, (int64_t)ray_colour_param_count(cfg->cmlp_width, cfg->cmlp_depth) * P, st));
  if (cfg->color_mode == 1 || cfg->color_mode == 3) {
    SNP_HIP(zero_f32(g->cmlp, (int64_t)cmlp_param_count(cfg->cmlp_width, cfg->cmlp_depth, cfg->color_mode == 3) * P,
                     st));
    SNP_HIP(zero_f32(g->xi, (int64_t)kXiDim * P, st));
  }
  if (cfg->color_mode == 2) SNP_HIP(zero_f32(g->sh, (int64_t)kShCoeffs * P, st));
  if (cfg->color_mode == 2) SNP_HIP(zero_f32(g->sh_t, (int64_t)kShTime * 3 * P, st));
  SNP_HIP(zero_f32(g->wt, N * P, st));
  return SNP_OK;
}

struct GraphHandle {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

// Captures `body` (a sequence of launches on the stream it is given) into a
// graph on a private non-blocking stream.
template <typename F>
static snp_status capture_graph(hipStream_t stream, void** graph_out, F body) {
  SNP_HIP(hipStreamSynchronize(stream));
  hipStream_t cs;
  SNP_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  GraphHandle* h = new GraphHandle();
  snp_status s = SNP_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) {
    s = SNP_ERR_HIP;
  } else {
    s = body(cs);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    if (s == SNP_OK && e != hipSuccess) s = SNP_ERR_HIP;
    if (s == SNP_OK) {
      h->graph = g;
      if (hipGraphInstantiate(&h->exec, g, nullptr, nullptr, 0) != hipSuccess) s = SNP_ERR_HIP;
    } else if (g) {
      (void)hipGraphDestroy(g);
    }
  }
  (void)hipStreamDestroy(cs);
  if (s != SNP_OK) {
    delete h;
    return s;
  }
  *graph_out = h;
  return SNP_OK;
}

#define SNP_TRY(x)                  \
  do {                              \
    snp_status s_ = (x);            \
    if (s_ != SNP_OK) return s_;    \
  } while (0)

// ---------------------------------------------------------------------------
// Static scratch of snp_step_static, for callers that cannot allocate device
// memory.  The array holds the whole workspace of one step.  On the host its
// name is only a stand-in symbol, never a device address: host code uses the
// address hipGetSymbolAddress returns, fetched once per device (every device
// holds its own copy of the array at its own address).
// ---------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[kMaxDevices];

static snp_status static_scratch(void** out) {
  int dev = -1;
  SNP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return SNP_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SNP_ERR_HIP;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return SNP_OK;
}

// The plan with the largest instance capacity whose workspace fits in the
// static scratch (the layout grows monotonically with the capacity).
static snp_status static_plan(const snp_config* cfg, int64_t P, int32_t V, const snp_camera* cams, Plan* pl) {
  SNP_TRY(make_plan(cfg, P, V, cams, 1, pl));
  if (pl->L.bytes > kStaticScratchBytes) return SNP_ERR_TOO_LARGE;
  int64_t lo = 1, hi = ((int64_t)1 << 31) - 1;
  Plan probe;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    SNP_TRY(make_plan(cfg, P, V, cams, mid, &probe));
    if (probe.L.bytes <= kStaticScratchBytes)
      lo = mid;
    else
      hi = mid - 1;
  }
  return make_plan(cfg, P, V, cams, lo, pl);
}

__global__ void copy_counters_kernel(const unsigned long long* src, int64_t* dst) {
  if (threadIdx.x < CNT_COUNT) dst[threadIdx.x] = (int64_t)src[threadIdx.x];
}

}  // namespace snp

using namespace snp;

extern "C" {

snp_status snp_workspace_layout(const snp_config* cfg, int64_t P, int32_t V, const snp_camera* cams,
                                int64_t max_instances, snp_layout* out) {
  if (!out) return SNP_ERR_INVALID;
  Plan pl;
  SNP_TRY(make_plan(cfg, P, V, cams, max_instances, &pl));
  *out = pl.L;
  return SNP_OK;
}

static bool same_layout(const snp_layout& a, const snp_layout& b) {
  return a.bytes == b.bytes && a.cams == b.cams && a.table == b.table && a.records == b.records &&
         a.rects == b.rects && a.depth_bits == b.depth_bits && a.tile_counts == b.tile_counts &&
         a.offsets == b.offsets && a.keys == b.keys && a.values == b.values && a.ranges == b.ranges &&
         a.counters == b.counters && a.gview == b.gview && a.gtable == b.gtable && a.loss == b.loss &&
         a.disc_coef == b.disc_coef &&
         a.capacity == b.capacity && a.table_stride == b.table_stride && a.total_tiles == b.total_tiles &&
         a.ahat_cache == b.ahat_cache && a.ahat_cache_bytes == b.ahat_cache_bytes && a.tile_pairs == b.tile_pairs;
}

// Rebuilds the plan of a call from its arguments and checks it against the
// caller's layout and workspace.
static snp_status plan_for(const snp_config* cfg, int64_t P, int32_t V, const snp_camera* cams, void* ws,
                           const snp_layout* layout, Plan* pl) {
  if (!layout) return SNP_ERR_INVALID;
  SNP_TRY(make_plan(cfg, P, V, cams, layout->capacity, pl));
  if (!same_layout(pl->L, *layout)) return SNP_ERR_INVALID;
  return check_ws(*pl, ws, layout->bytes);
}

snp_status snp_preprocess(const snp_config* cfg, const snp_prims* prims, int32_t V, const snp_camera* cams, void* ws,
                          const snp_layout* layout, hipStream_t stream) {
  if (!cfg || !prims) return SNP_ERR_INVALID;
  Plan pl;
  SNP_TRY(plan_for(cfg, prims->P, V, cams, ws, layout, &pl));
  SNP_TRY(check_prims(cfg, prims));
  return do_preprocess(cfg, prims, V, cams, pl, ws, stream);
}

snp_status snp_bin(const snp_config* cfg, int64_t P, int32_t V, const snp_camera* cams, void* ws,
                   const snp_layout* layout, hipStream_t stream) {
  Plan pl;
  SNP_TRY(plan_for(cfg, P, V, cams, ws, layout, &pl));
  return do_bin(cfg, P, V, pl, ws, stream);
}

snp_status snp_sort(const snp_config* cfg, int64_t P, int32_t V, const snp_camera* cams, void* ws,
                    const snp_layout* layout, hipStream_t stream) {
  Plan pl;
  SNP_TRY(plan_for(cfg, P, V, cams, ws, layout, &pl));
  return do_sort(pl, ws, stream);
}

snp_status snp_render_forward(const snp_config* cfg, const snp_prims* prims, int32_t V, const snp_camera* cams,
                              void* ws, const snp_layout* layout, float* images, float* final_T, int32_t count_pairs,
                              hipStream_t stream) {
  if (!cfg || !prims || !images || !final_T) return SNP_ERR_INVALID;
  Plan pl;
  SNP_TRY(plan_for(cfg, prims->P, V, cams, ws, layout, &pl));
  SNP_TRY(check_prims(cfg, prims));
  return do_forward(cfg, prims->P, V, pl, ws, images, final_T, count_pairs, stream);
}

static snp_status do_loss(const Plan& pl, const float* images, const float* targets, double n_norm, void* ws,
                          double* loss_out, float* dL, hipStream_t st) {
  SNP_HIP(launch_l1(images, targets, 3 * pl.total_pixels, n_norm, dL, wsp<double>(ws, pl.L.loss), loss_out, st));
  return SNP_OK;
}

snp_status snp_loss_l1(const snp_config* cfg, int32_t V, const snp_camera* cams, const float* images,
                       const float* targets, double n_norm, void* ws, const snp_layout* layout, double* loss_out,
                       float* dL_dimages, hipStream_t stream) {
  if (!images || !targets || !loss_out || !dL_dimages || !(n_norm > 0.0) || !layout) return SNP_ERR_INVALID;
  SNP_TRY(check_cfg(cfg));
  SNP_TRY(check_cams(V, cams));
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0 || layout->loss + loss_scratch_bytes() > layout->bytes)
    return SNP_ERR_INVALID;
  Plan pl;
  pl.L = *layout;
  pl.total_pixels = 0;
  for (int v = 0; v < V; ++v) pl.total_pixels += (int64_t)cams[v].width * cams[v].height;
  return do_loss(pl, images, targets, n_norm, ws, loss_out, dL_dimages, stream);
}

snp_status snp_render_backward(const snp_config* cfg, const snp_prims* prims, int32_t V, const snp_camera* cams,
                               void* ws, const snp_layout* layout, const float* images, const float* dL_dimages,
                               const snp_grads* grads, hipStream_t stream) {
  if (!cfg || !prims || !images || !dL_dimages || !grads) return SNP_ERR_INVALID;
  if (gaussian(cfg)) return SNP_ERR_UNSUPPORTED;
  Plan pl;
  SNP_TRY(plan_for(cfg, prims->P, V, cams, ws, layout, &pl));
  SNP_TRY(check_prims(cfg, prims));
  return do_backward(cfg, prims, V, pl, ws, images, dL_dimages, grads, stream);
}

static snp_status do_step(const snp_config* cfg, const snp_prims* prims, int32_t V, const snp_camera* cams,
                          const Plan& pl, void* ws, float* images, float* final_T, const float* targets,
                          double n_norm, double* loss_out, float* dL, const snp_grads* grads, hipStream_t st) {
  SNP_TRY(zero_grads(cfg, prims->P, grads, st));
  SNP_TRY(do_preprocess(cfg, prims, V, cams, pl, ws, st));
  SNP_TRY(do_bin(cfg, prims->P, V, pl, ws, st));
  SNP_TRY(do_sort(pl, ws, st));
  SNP_TRY(do_forward(cfg, prims->P, V, pl, ws, images, final_T, 0, st));
  SNP_TRY(do_loss(pl, images, targets, n_norm, ws, loss_out, dL, st));
  SNP_TRY(do_backward(cfg, prims, V, pl, ws, images, dL, grads, st));
  return SNP_OK;
}

static snp_status check_step_args(const snp_config* cfg, const snp_prims* prims, float* images, float* final_T,
                                  const float* targets, double n_norm, double* loss_out, float* dL,
                                  const snp_grads* grads) {
  if (!cfg || !prims || !images || !final_T || !targets || !loss_out || !dL || !grads || !(n_norm > 0.0))
    return SNP_ERR_INVALID;
  if (gaussian(cfg)) return SNP_ERR_UNSUPPORTED;
  return check_prims(cfg, prims);
}

snp_status snp_step(const snp_config* cfg, const snp_prims* prims, int32_t V, const snp_camera* cams, void* ws,
                    const snp_layout* layout, float* images, float* final_T, const float* targets, double n_norm,
                    double* loss_out, float* dL_dimages, const snp_grads* grads, hipStream_t stream) {
  SNP_TRY(check_step_args(cfg, prims, images, final_T, targets, n_norm, loss_out, dL_dimages, grads));
  Plan pl;
  SNP_TRY(plan_for(cfg, prims->P, V, cams, ws, layout, &pl));
  return do_step(cfg, prims, V, cams, pl, ws, images, final_T, targets, n_norm, loss_out, dL_dimages, grads, stream);
}

snp_status snp_step_static(const snp_config* cfg, const snp_prims* prims, int32_t V, const snp_camera* cams,
                           float* images, float* final_T, const float* targets, double n_norm, double* loss_out,
                           float* dL_dimages, const snp_grads* grads, int64_t* counters_out, hipStream_t stream) {
  SNP_TRY(check_step_args(cfg, prims, images, final_T, targets, n_norm, loss_out, dL_dimages, grads));
  Plan pl;
  SNP_TRY(static_plan(cfg, prims->P, V, cams, &pl));
  void* ws = nullptr;
  SNP_TRY(static_scratch(&ws));
  SNP_TRY(do_step(cfg, prims, V, cams, pl, ws, images, final_T, targets, n_norm, loss_out, dL_dimages, grads, stream));
  if (counters_out) {
    hipLaunchKernelGGL(copy_counters_kernel, dim3(1), dim3(64), 0, stream, wsp<unsigned long long>(ws, pl.L.counters),
                       counters_out);
    SNP_HIP(hipGetLastError());
  }
  return SNP_OK;
}

snp_status snp_graph_create(const snp_config* cfg, const snp_prims* prims, int32_t V, const snp_camera* cams,
                            void* ws, const snp_layout* layout, float* images, float* final_T, const float* targets,
                            double n_norm, double* loss_out, float* dL_dimages, const snp_grads* grads,
                            hipStream_t stream, void** graph_out) {
  if (!graph_out) return SNP_ERR_INVALID;
  SNP_TRY(check_step_args(cfg, prims, images, final_T, targets, n_norm, loss_out, dL_dimages, grads));
  Plan pl;
  SNP_TRY(plan_for(cfg, prims->P, V, cams, ws, layout, &pl));
  return capture_graph(stream, graph_out, [&](hipStream_t cs) {
    return do_step(cfg, prims, V, cams, pl, ws, images, final_T, targets, n_norm, loss_out, dL_dimages, grads, cs);
  });
}

snp_status snp_graph_create_forward(const snp_config* cfg, const snp_prims* prims, int32_t V,
                                    const snp_camera* cams, void* ws, const snp_layout* layout, float* images,
                                    float* final_T, hipStream_t stream, void** graph_out) {
  if (!graph_out || !cfg || !prims || !images || !final_T) return SNP_ERR_INVALID;
  Plan pl;
  SNP_TRY(plan_for(cfg, prims->P, V, cams, ws, layout, &pl));
  SNP_TRY(check_prims(cfg, prims));
  return capture_graph(stream, graph_out, [&](hipStream_t cs) {
    SNP_TRY(do_preprocess(cfg, prims, V, cams, pl, ws, cs));
    SNP_TRY(do_bin(cfg, prims->P, V, pl, ws, cs));
    SNP_TRY(do_sort(pl, ws, cs));
    return do_forward(cfg, prims->P, V, pl, ws, images, final_T, 0, cs);
  });
}

snp_status snp_graph_launch(void* graph, hipStream_t stream) {
  if (!graph) return SNP_ERR_INVALID;
  GraphHandle* h = reinterpret_cast<GraphHandle*>(graph);
  SNP_HIP(hipGraphLaunch(h->exec, stream));
  return SNP_OK;
}

snp_status snp_graph_destroy(void* graph) {
  if (!graph) return SNP_ERR_INVALID;
  GraphHandle* h = reinterpret_cast<GraphHandle*>(graph);
  (void)hipGraphExecDestroy(h->exec);
  (void)hipGraphDestroy(h->graph);
  delete h;
  return SNP_OK;
}

snp_status snp_read_counters(void* ws, const snp_layout* layout, int64_t* out8, hipStream_t stream) {
  if (!ws || !layout || !out8) return SNP_ERR_INVALID;
  SNP_HIP(hipStreamSynchronize(stream));
  unsigned long long c[CNT_COUNT];
  SNP_HIP(hipMemcpy(c, reinterpret_cast<char*>(ws) + layout->counters, sizeof(c), hipMemcpyDeviceToHost));
  for (int i = 0; i < CNT_COUNT; ++i) out8[i] = (int64_t)c[i];
  return SNP_OK;
}

snp_status snp_read_status(void* ws, const snp_layout* layout, int64_t* instances_out, int64_t* hit_pairs_out,
                           hipStream_t stream) {
  if (!ws || !layout) return SNP_ERR_INVALID;
  SNP_HIP(hipStreamSynchronize(stream));
  unsigned long long c[CNT_COUNT];
  SNP_HIP(hipMemcpy(c, reinterpret_cast<char*>(ws) + layout->counters, sizeof(c), hipMemcpyDeviceToHost));
  if (instances_out) *instances_out = (int64_t)c[CNT_INSTANCES];
  if (hit_pairs_out) *hit_pairs_out = (int64_t)c[CNT_HIT_PAIRS];
  if (c[CNT_OVERFLOW]) return SNP_ERR_CAPACITY;
  if (c[CNT_RANGE]) return SNP_ERR_RANGE;
  return SNP_OK;
}

int32_t snp_supported_tiles(int32_t* triples, int32_t max) {
  if (!triples) max = 0;
  return supported_tiles(triples, max);
}

const char* snp_status_string(snp_status s) {
  switch (s) {
    case SNP_OK: return "ok";
    case SNP_ERR_INVALID: return "invalid argument";
    case SNP_ERR_CAPACITY: return "tile instances exceeded the workspace capacity";
    case SNP_ERR_HIP: return "HIP runtime error";
    case SNP_ERR_UNSUPPORTED: return "unsupported configuration";
    case SNP_ERR_RANGE: return "density-MLP phase outside the supported range";
    case SNP_ERR_TOO_LARGE: return "the step does not fit in the 64 MiB static scratch";
  }
  return "unknown status";
}

snp_status snp_kernel_timing(int32_t enable) {
  if (enable && !g_timer.e[0])
    for (int i = 0; i < 4; ++i) SNP_HIP(hipEventCreate(&g_timer.e[i]));
  g_timer.on = enable != 0;
  g_timer.have_fwd = g_timer.have_bwd = false;
  return SNP_OK;
}

snp_status snp_kernel_timing_read(float* fwd_ms, float* bwd_ms) {
  if (!fwd_ms || !bwd_ms) return SNP_ERR_INVALID;
  *fwd_ms = *bwd_ms = -1.f;
  if (g_timer.have_fwd) {
    SNP_HIP(hipEventSynchronize(g_timer.e[1]));
    SNP_HIP(hipEventElapsedTime(fwd_ms, g_timer.e[0], g_timer.e[1]));
  }
  if (g_timer.have_bwd) {
    SNP_HIP(hipEventSynchronize(g_timer.e[3]));
    SNP_HIP(hipEventElapsedTime(bwd_ms, g_timer.e[2], g_timer.e[3]));
  }
  return SNP_OK;
}

snp_status snp_adam_step(const snp_adam_group* groups, int32_t n_groups, int64_t step, double beta1, double beta2,
                         double eps, hipStream_t stream) {
  if (!groups || n_groups < 0 || n_groups > SNP_MAX_ADAM_GROUPS || step < 1) return SNP_ERR_INVALID;
  if (!(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0 && eps >= 0.0)) return SNP_ERR_INVALID;
  for (int k = 0; k < n_groups; ++k) {
    const snp_adam_group& g = groups[k];
    if (g.n < 0) return SNP_ERR_INVALID;
    if (g.n > 0 && (!g.param || !g.grad || !g.m || !g.v)) return SNP_ERR_INVALID;
    if (g.log_space != 0 && g.log_space != 1) return SNP_ERR_INVALID;
  }
  SNP_HIP(launch_adam(groups, n_groups, step, beta1, beta2, eps, stream));
  return SNP_OK;
}

static bool loss_scratch_ok(void* ws, const snp_layout* layout) {
  return ws && layout && (reinterpret_cast<uintptr_t>(ws) & 255) == 0 &&
         layout->loss + loss_scratch_bytes() <= layout->bytes;
}

snp_status snp_scale_regularizer(int64_t P, const float* scales, float weight, float* grad_scales, double* loss_out,
                                 void* ws, const snp_layout* layout, hipStream_t stream) {
  if (P <= 0 || !scales || !loss_out || !std::isfinite(weight) || !loss_scratch_ok(ws, layout)) return SNP_ERR_INVALID;
  SNP_HIP(launch_scale_reg(P, scales, weight, grad_scales, wsp<double>(ws, layout->loss), loss_out, stream));
  return SNP_OK;
}

snp_status snp_densify_accumulate(int64_t P, int32_t N, int32_t V, const snp_grads* grads, void* ws,
                                  const snp_layout* layout, float* grad_acc, float* visible, hipStream_t stream) {
  if (P <= 0 || V <= 0 || N <= 0 || !grads || !grads->w1 || !grads->b1 || !grads->w2 || !grads->b2 || !ws ||
      !layout || !grad_acc || !visible)
    return SNP_ERR_INVALID;
  if (layout->tile_counts + sizeof(uint32_t) * (size_t)V * (size_t)P > layout->bytes) return SNP_ERR_INVALID;
  SNP_HIP(launch_densify_acc(P, N, V, *grads, wsp<uint32_t>(ws, layout->tile_counts), grad_acc, visible, stream));
  return SNP_OK;
}

size_t snp_densify_scratch_bytes(int64_t P) { return P > 0 ? densify_scratch_bytes(P) : 0; }

snp_status snp_densify_plan(int64_t P, const float* scales, const float* grad_acc, const float* visible,
                            const snp_density_control* dc, int32_t* action, uint32_t* offsets, int64_t* new_count,
                            void* scratch, size_t scratch_bytes, hipStream_t stream) {
  if (P <= 0 || P > ((int64_t)1 << 31) - 1 || !scales || !grad_acc || !visible || !dc || !action || !offsets ||
      !new_count || !scratch || scratch_bytes < densify_scratch_bytes(P))
    return SNP_ERR_INVALID;
  SNP_HIP(launch_densify_plan(P, scales, grad_acc, visible, *dc, action, offsets, new_count, scratch, stream));
  return SNP_OK;
}

snp_status snp_densify_apply(int64_t P, const int32_t* action, const uint32_t* offsets, const float* centers,
                             const float* scales, const float* quats, const float* noise, float split_shrink,
                             const snp_row_array* arrays, int32_t n_arrays, hipStream_t stream) {
  if (P <= 0 || !action || !offsets || !arrays || n_arrays < 0 || !(split_shrink > 0.f)) return SNP_ERR_INVALID;
  for (int k = 0; k < n_arrays; ++k) {
    const snp_row_array& a = arrays[k];
    if (!a.src || !a.dst || a.width <= 0 || a.kind < SNP_ROWS_PARAM || a.kind > SNP_ROWS_SCALES)
      return SNP_ERR_INVALID;
    if (a.kind == SNP_ROWS_CENTERS && (a.width != 3 || !centers || !scales || !quats || !noise))
      return SNP_ERR_INVALID;
    if (a.kind == SNP_ROWS_SCALES && a.width != 3) return SNP_ERR_INVALID;
  }
  for (int k = 0; k < n_arrays; ++k)
    SNP_HIP(launch_densify_apply(P, action, offsets, centers, scales, quats, noise, split_shrink, arrays[k], stream));
  return SNP_OK;
}

snp_status snp_selftest_wave_sum(const float* in, float* out, int32_t waves, hipStream_t stream) {
  if (!in || !out || waves <= 0) return SNP_ERR_INVALID;
  SNP_HIP(launch_wave_sum_selftest(in, out, waves, stream));
  return SNP_OK;
}

}  // extern "C"
