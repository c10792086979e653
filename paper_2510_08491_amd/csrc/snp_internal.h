// Internal layouts and device helpers shared by the kernels of libsnp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "../../include/snp.h"

namespace snp {

constexpr float kTwoPi = 6.283185307179586f;
constexpr float kInvTwoPi = 0.15915494309189535f;
constexpr float kLog2e = 1.4426950408889634f;
constexpr double kEpsPx = 1.0 / 64.0;  // slack of the pixel rectangle, in pixels
constexpr int kRecFloats = 24;         // per-(view, primitive) record
constexpr int kGViewFloats = 24;       // per-(view, primitive) gradient record
constexpr int kMaxCamsPerChunk = 16;   // cameras passed by value per launch
constexpr int kXiDim = 8;
constexpr int kCmlpIn = 3 + kXiDim;
constexpr int kShCoeffs = 48;     // spherical harmonics of degree 3: 16 basis functions x RGB
constexpr int kRayIn = 9;         // per-ray relighting colour: entry point, ray direction, light direction

// Per-ray relighting colour (colour mode 4), width W, D hidden layers.  The
// network's parameters per primitive (cmlp): W1 (W x 9) over [entry point
// (x - x_B)/m, ray direction d, light direction], b1, [Wh (W x W), bh],
// Wo (3 x W), bo.  The rasterizer evaluates it from a per-primitive table in
// the ellipsoid's unit-sphere frame (u = S^-1 R^T (x - x_B), d' the ray
// direction in that frame, L the length of the un-normalised camera ray):
//   W1[:, 0:3] (x - x_B)/m = Au u,   Au = W1[:, 0:3] R S / m
//   W1[:, 3:6] d           = Ad d' / L,   Ad = W1[:, 3:6] R S
// and a per-(view, primitive) bias cb = b1 + W1[:, 6:9] normalize(l_v - x_B).
// Table row: Au (k*3 + j), Ad, [Wh, bh], Wo, bo, padded to a multiple of 4.
template <int W, int D>
struct RayColourLayout {
  static constexpr int AU = 0;
  static constexpr int AD = 3 * W;
  static constexpr int WH = 6 * W;
  static constexpr int BH = WH + W * W;
  static constexpr int WO = D == 2 ? BH + W : 6 * W;
  static constexpr int BO = WO + 3 * W;
  static constexpr int CT = BO + 3;
  static constexpr int CTS = (CT + 3) / 4 * 4;  // row stride
};
inline __host__ __device__ int ray_colour_stride(int W, int D) {
  return ((6 * W + (D == 2 ? W * W + W : 0) + 3 * W + 3) + 3) / 4 * 4;
}

// Per-view constants on the device.
struct CamDev {
  int32_t width, height, ntx, nty;
  int32_t tile_base;  // global id of the view's first tile
  int32_t tile_w, tile_h, pad0;
  int64_t pix_base;   // index of the view's first pixel in the packed images
  float fx, fy, cx, cy;
  float R[9];
  float t[3];
  float Rinv_f[9];    // camera -> world, float copy for per-pixel directions
  float o_f[3];
  float light[3];     // the view's point light (relighting colour)
  double Rinv[9];     // camera -> world (exact inverse of R, float64)
  double o[3];        // camera centre -R^-1 t
};

struct CamChunk {  // kernel argument carrying up to kMaxCamsPerChunk cameras
  snp_camera cam[kMaxCamsPerChunk];
  int32_t tile_base[kMaxCamsPerChunk];
  int64_t pix_base[kMaxCamsPerChunk];
  int32_t first, count, tile_w, tile_h;
};

// Counters at layout.counters (uint64 each).
enum Counter {
  CNT_INSTANCES = 0,
  CNT_OVERFLOW = 1,
  CNT_HIT_PAIRS = 2,
  CNT_RANGE = 3,
  CNT_QUEUE_FWD = 4,
  CNT_QUEUE_BWD = 5,
  CNT_LIVE_PAIRS = 6,
  CNT_DEPTH_SORT = 7,  // number of (view, primitive) pairs, the length of the depth sort
  CNT_COUNT = 8
};

// Table row of a primitive, TS = 5N + 4 floats:
//   [4k .. 4k+3]   (Wt_k.x, Wt_k.y, Wt_k.z, bt_k)  phase coefficients in revolutions
//   [4N + k]       W2_k / (2 pi)
//   [5N]           b2
inline __host__ __device__ int table_stride(int N) { return 5 * N + 4; }

// Record of a Gaussian (view, primitive) pair uses q2..q4 only (the colour
// stays where the colour kernels write it):
//   q2 (u, v, ka, col.r)  q3 (kb, kc, opacity, col.g)  q4 (0, 0, 0, col.b)
// with (u, v) the projected centre in pixels and, for the pixel offset
// (dx, dy) = pixel centre - (u, v), log2 of the Gaussian factor
//   ka dx^2 + kb dx dy + kc dy^2   (<= 0)
//
// Record of a (view, primitive) pair, 6 float4:
//   q0 (dc.xyz, rx)  q1 (gx.xyz, ry)  q2 (gy.xyz, col.r)
//   q3 (mc.xyz, col.g)  q4 (hx.xyz, col.b)  q5 (hy.xyz, band)
// For a pixel centre (px, py), with dx = px - rx, dy = py - ry:
//   d' = dc + gx dx + gy dy   ray direction in the ellipsoid's unit-sphere frame
//   m' = mc + hx dx + hy dy   its moment o' x d'
// where the direction is the un-normalised camera ray R^-1 (x, y, 1).
// The discriminant A - M = |d'|^2 - |m'|^2 as a float64 quadratic form in the
// same offsets is kept beside the record (6 doubles c0..c5):
//   disc = c0 + dx (c1 + c3 dx + c4 dy) + dy (c2 + c5 dy)
// Where the float32 difference A - M lies within `band` of zero (64 times a
// bound on its rounding error over the rectangle) its sign is not trusted
// and the float64 form decides the hit and gives the value; the gradient
// phase of the backward also takes the float64 value within 1% of A of
// zero, where the float32 difference has too few correct digits for the
// 1/sqrt(disc) factor of the geometry gradient.

template <typename T>
__device__ __forceinline__ T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off);
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
// sin / cos of 2 pi x (x in revolutions, |x| <= 256)
__device__ __forceinline__ float sin_rev(float x) { return __builtin_amdgcn_sinf(x); }
__device__ __forceinline__ float cos_rev(float x) { return __builtin_amdgcn_cosf(x); }
__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }

__device__ __forceinline__ float wave_sum(float v) {
  // butterfly over the 64 lanes; every lane ends with the total
  v += __shfl_xor(v, 1);
  v += __shfl_xor(v, 2);
  v += __shfl_xor(v, 4);
  v += __shfl_xor(v, 8);
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

__device__ __forceinline__ void atomic_add_f32(float* p, float v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Global tile id -> view index (V small; linear scan over tile bases).
__device__ __forceinline__ int view_of_tile(const CamDev* cams, int V, int gtile) {
  int v = 0;
  while (v + 1 < V && cams[v + 1].tile_base <= gtile) ++v;
  return v;
}

}  // namespace snp

// ---------------------------------------------------------------------------
// kernel arguments and host launchers (implemented in the .hip files)
// ---------------------------------------------------------------------------
namespace snp {

struct ViewArgs {
  int64_t P;
  int32_t V;
  float z_near;
  int32_t color_mode;
  int32_t primitive;  // 0 neural, 1 Gaussian
  const float *centers, *scales, *quats, *colors;
  const float* opacity;
  const CamDev* cams;
  float* records;
  int32_t* rects;
  uint32_t* depth_bits;
  uint32_t* tile_counts;
  double* disc_coef;
};

struct CmlpArgs {
  int64_t P;
  int32_t V;
  int32_t relight;  // 1: relighting colour (light direction input, plus c_dc = colors)
  const float *centers, *xi, *cmlp, *colors;
  const CamDev* cams;
  const uint32_t* tile_counts;
  float* records;
  float* gview;
  float* g_cmlp;
  float* g_xi;
  float* g_centers;  // relighting: the light direction's chain to the centres
};

constexpr int kShTime = 12;  // time-dependent zero-order SH: xi^1..4, cos(i xi), sin(i xi), i = 1..4

struct ShArgs {
  int64_t P;
  int32_t V;
  const float *centers, *sh;
  const float* sh_t;       // P x 12 x 3 time coefficients of the zero-order term, or null
  float tb[kShTime];       // the 12 functions of xi_t they multiply
  const CamDev* cams;
  const uint32_t* tile_counts;
  float* records;
  float* gview;
  float* g_sh;
  float* g_sh_t;
};

struct PreBwdArgs {
  int64_t P;
  int32_t V, N, color_mode;
  float omega0, time;
  const float *centers, *scales, *quats, *w1;
  const CamDev* cams;
  const float* records;
  const uint32_t* tile_counts;
  const float* gview;
  const float* gtable;
  const float* extra_rs;  // per primitive 12 floats: further d loss / d R (9) and d loss / d s (3), or null
  snp_grads g;
};

// per-ray relighting colour (colour mode 4): the preprocess side
struct RayColourArgs {
  int64_t P;
  int32_t V, W, D;
  const float *centers, *scales, *quats, *cmlp;
  const CamDev* cams;
  const uint32_t* tile_counts;
  float* ctab;          // P x stride: the network in the unit-sphere frame
  float* cbias;         // V P x W: first-layer bias with the light term
  const float* gctab;   // backward: gradient of ctab
  const float* gcbias;  // backward: gradient of cbias
  float* g_cmlp;
  float* g_centers;
  float* extra_rs;      // backward: per primitive d loss / d R (9), d loss / d s (3) for the preprocess adjoint
};

struct EmitArgs {
  int64_t P;
  int32_t V;
  int64_t capacity;
  const CamDev* cams;
  const int32_t* rects;
  const uint32_t* depth_bits;
  const uint32_t* tile_counts;
  const uint32_t* order;    // (view, primitive) pair indices in depth order
  const uint32_t* offsets;  // first instance of each pair, in depth order
  unsigned long long* keys;
  uint32_t* values;
};

struct RasterArgs {
  const CamDev* cams;
  int32_t V;
  int64_t P;
  int32_t total_tiles;
  const float* table;
  const float* records;
  const uint32_t* values;
  const uint32_t* ranges;
  const uint32_t* tile_order;  // persistent launches: tiles by instance count, descending (null: in id order)
  const int32_t* rects;   // per (view, primitive) pixel rectangle x0, x1, y0, y1
  float* images;          // forward output
  float* final_T;         // forward output
  const float* images_in; // backward: forward's images
  const float* dL;        // backward: d loss / d images
  float* gview;
  float* gtable;
  const double* disc_coef;  // float64 discriminant coefficients: hit decisions near silhouettes
  int64_t cache_instances;  // leading instances covered by ahat_cache
  float* ahat_cache;        // per (instance, tile pixel) integral: the forward writes it,
                            // the backward reads it (null: the backward re-evaluates)
  const float* ctab;        // colour mode 4: per-primitive colour network table
  const float* cbias;       // colour mode 4: per-(view, primitive) first-layer bias
  float* gctab;             // colour mode 4 backward: gradients of ctab, cbias
  float* gcbias;
  unsigned long long* counters;
  uint32_t* tile_pairs;     // forward with pair counting: hit pairs per global tile
  float t_eps, alpha_min, alpha_max;
  float bg0, bg1, bg2;
};

// preprocess.hip
hipError_t launch_setup_cams(const CamChunk& ch, CamDev* out, hipStream_t st);
hipError_t launch_prim_table(int N, int64_t P, float omega0, float time, const snp_prims& pr, float* table,
                             unsigned long long* counters, hipStream_t st);
hipError_t launch_preprocess_views(const ViewArgs& a, hipStream_t st);
hipError_t launch_cmlp_fwd(int width, int depth, CmlpArgs a, hipStream_t st);
hipError_t launch_cmlp_bwd(int width, int depth, CmlpArgs a, hipStream_t st);
// sh.hip
hipError_t launch_sh_fwd(const ShArgs& a, hipStream_t st);
hipError_t launch_sh_bwd(const ShArgs& a, hipStream_t st);
bool cmlp_supported(int width, int depth);
int cmlp_param_count(int width, int depth, bool relight);
hipError_t launch_preprocess_bwd(const PreBwdArgs& a, hipStream_t st);
// relight.hip
bool ray_colour_supported(int width, int depth);
int ray_colour_param_count(int width, int depth);
hipError_t launch_ray_colour_fwd(const RayColourArgs& a, hipStream_t st);
hipError_t launch_ray_colour_bwd(const RayColourArgs& a, hipStream_t st);
// binning.hip
hipError_t fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);
size_t scan_scratch_bytes(int64_t n);
hipError_t scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, void* scratch, uint64_t* total_out,
                              hipStream_t st);
hipError_t launch_emit(const EmitArgs& a, unsigned long long* counters, hipStream_t st);
size_t sort_scratch_bytes(int64_t capacity);
hipError_t radix_sort(unsigned long long* k0, uint32_t* v0, unsigned long long* k1, uint32_t* v1, int64_t capacity,
                      const unsigned long long* count, int lo_bit, int key_bits, void* scratch, hipStream_t st);
hipError_t launch_depth_keys(const uint32_t* depth_bits, int64_t n, unsigned long long* keys, uint32_t* idx,
                             unsigned long long* n_out, hipStream_t st);
hipError_t launch_gather_counts(const uint32_t* order, const uint32_t* counts, int64_t n, uint32_t* out,
                                hipStream_t st);
int radix_passes(int key_bits);
hipError_t launch_ranges(const unsigned long long* keys, const unsigned long long* counters, int64_t capacity,
                         uint32_t* ranges, int64_t n_tiles, hipStream_t st);
hipError_t launch_tile_keys(const uint32_t* ranges, int64_t n_tiles, unsigned long long* keys, uint32_t* ids,
                            unsigned long long* n_out, hipStream_t st);
// raster.hip
int supported_tiles(int32_t* triples, int32_t max);
bool tile_supported(int tw, int th, int ppl);
bool bwd_batch_supported(int tw, int th, int nb);
bool ray_colour_raster_supported(int N, int tw, int th, int ppl, int nb);
int bwd_batch_default(int tw, int th);
// cd: 0, or the depth of the per-ray colour network (colour mode 4, width 16)
hipError_t launch_render_fwd(int N, int tw, int th, int ppl, bool persist, bool count, int cd, const RasterArgs& a,
                             hipStream_t st);
hipError_t launch_render_bwd(int N, int tw, int th, int nb, bool persist, int cd, const RasterArgs& a,
                             hipStream_t st);
hipError_t launch_render_fwd_gauss(int tw, int th, int ppl, bool persist, bool count, const RasterArgs& a,
                                   hipStream_t st);
hipError_t launch_wave_sum_selftest(const float* in, float* out, int waves, hipStream_t st);
// train.hip
hipError_t launch_adam(const snp_adam_group* groups, int ng, int64_t step, double b1, double b2, double eps,
                       hipStream_t st);
hipError_t launch_scale_reg(int64_t P, const float* scales, float weight, float* grad, double* partials,
                            double* loss_out, hipStream_t st);
hipError_t launch_densify_acc(int64_t P, int N, int V, const snp_grads& g, const uint32_t* tile_counts, float* acc,
                              float* cnt, hipStream_t st);
size_t densify_scratch_bytes(int64_t P);
hipError_t launch_densify_plan(int64_t P, const float* scales, const float* acc, const float* cnt,
                               const snp_density_control& dc, int32_t* action, uint32_t* offsets, int64_t* new_count,
                               void* scratch, hipStream_t st);
hipError_t launch_densify_apply(int64_t P, const int32_t* action, const uint32_t* offsets, const float* centers,
                                const float* scales, const float* quats, const float* noise, float shrink,
                                const snp_row_array& arr, hipStream_t st);
// loss.hip
size_t loss_scratch_bytes();
hipError_t launch_l1(const float* img, const float* tgt, int64_t n, double n_norm, float* grad, double* partials,
                     double* out, hipStream_t st);
hipError_t zero_f32(float* p, int64_t n, hipStream_t st);
hipError_t zero_counters(unsigned long long* p, int n, hipStream_t st);
hipError_t zero_counter(unsigned long long* p, hipStream_t st);

}  // namespace snp
