// Tile rasterizer of neural primitives: forward (Eq. 3-4, 7-9) and adjoint.
//
// A workgroup renders one tile (TW x TH pixels, PPL pixels per thread, rows
// stacked, or 8 x 8 blocks per wave).  It walks the tile's depth-sorted
// instance list in batches of primitives; each batch's records (24 floats per (view, primitive))
// and density tables (5N + 4 floats per primitive) are staged in LDS by the
// whole workgroup and then read as broadcasts.  Per pixel and primitive:
//
//   d' = dc + gx dx + gy dy,  m' = mc + hx dx + hy dy          (ray in B's frame)
//   A = |d'|^2, M = |m'|^2, disc = A - M;  hit iff disc > 0     (line-ellipsoid)
//   H = sqrt(disc)/A (half chord), p' = d' x m' / A (midpoint), e' = d' H
//   Q = b2 + sum_k W2_k cos(2 pi (Wt_k.p' + bt_k)) sinc(2 pi Wt_k.e')
//   integral = 2 L H Q   (L = length of the un-normalised ray direction)
//
// which is S(t_out) - S(t_in) of Eq. 8 rearranged around the chord midpoint
// (sin(u+v) - sin(u-v) = 2 cos u sin v); alpha = 1 - exp(-max(0, integral))
// (Eq. 9), then C += c alpha T, T *= 1 - alpha (Eq. 4).  A pixel stops taking
// primitives once T < t_eps; the workgroup leaves the list when every pixel
// has stopped.
//
// The adjoint walks the same list in the same order, recomputing T, and uses
// the final colour to get the colour of everything behind each primitive:
//   d loss / d integral = sum_c g_c (c_c T (1 - alpha) - behind_c)
// (behind = C_final - C_accumulated_after), so no per-pixel history is kept.
// Per-pair gradients of the table entries and of the record coefficients are
// summed over the wave with DPP and added to per-primitive / per-(view,
// primitive) accumulators with one atomic per value per wave.
#include "snp_internal.h"

namespace snp {

// instances per forward batch: 64, or 32 for N = 32 (whose tables would take
// most of the LDS at 64 and cut the occupancy), or 8 with the per-ray colour
// network (its table takes 1.7 KB per instance)
template <int N, int CD = 0>
constexpr int fwd_batch() { return CD > 0 ? 8 : (N >= 32 ? 32 : 64); }


// sum over the 64 lanes; the total ends in lane 63 (other lanes hold partials)
__device__ __forceinline__ float dpp_sum_last(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));  // row_half_mirror
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false));  // row_mirror
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xA, 0xF, false));  // row_bcast:15
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xC, 0xF, false));  // row_bcast:31
  return v;
}

__device__ __forceinline__ float wave_total(float v) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(dpp_sum_last(v)), 63));
}

// sinc(2 pi hv) * 2 pi = sin(2 pi hv) / hv.  The hardware sine keeps its
// relative accuracy (about 5e-7) down to the smallest arguments, so the
// product with 1/hv needs no small-argument branch; at hv = 0 it is 0 * inf
// = NaN, and the minimum with the limit 2 pi (which returns the non-NaN
// operand; sin(x)/x <= 2 pi everywhere) turns that into the limit.
__device__ __forceinline__ float sinc_rev(float s, float hv) { return fminf(s * fast_rcp(hv), kTwoPi); }

// Per-thread pixels of a tile.  With one pixel per thread and a tile of whole
// 8 x 8 blocks, each wave covers one 8 x 8 block (a compact footprint, so
// fewer waves are only partly covered by a primitive); otherwise a wave covers
// 64 / TW thread rows of TW pixels, PPL pixel rows per thread.  loc is the
// pixel's index in the tile (row-major), independent of the thread mapping.
template <int TW, int TH, int PPL>
struct PixelBlock {
  static_assert(64 % TW == 0 || (PPL == 1 && TW % 8 == 0), "a wave must cover whole tile rows or 8 x 8 blocks");
  static constexpr bool kBlocks = PPL == 1 && TW % 8 == 0 && TH % 8 == 0;
  float pxc[PPL], pyc[PPL], L[PPL];
  int pix[PPL];  // index into the packed image, -1 if outside
  int loc[PPL];  // index in the tile
  int wx0, wx1, wy0, wy1;  // pixel block of this thread's wave
  __device__ void init(const CamDev& cam, int tx, int ty) {
    int lx, ly0;
    if constexpr (kBlocks) {
      const int w = (int)(threadIdx.x / 64), l = (int)(threadIdx.x % 64);
      const int bx = w % (TW / 8), by = w / (TW / 8);
      lx = bx * 8 + l % 8;
      ly0 = by * 8 + l / 8;
      wx0 = tx * TW + bx * 8;
      wx1 = wx0 + 7;
      wy0 = ty * TH + by * 8;
      wy1 = wy0 + 7;
    } else {
      constexpr int ROWS = (64 / TW) * PPL;  // pixel rows covered by one wave
      wx0 = tx * TW;
      wx1 = wx0 + TW - 1;
      wy0 = ty * TH + (int)(threadIdx.x / 64) * ROWS;
      wy1 = wy0 + ROWS - 1;
      lx = threadIdx.x % TW;
      ly0 = (threadIdx.x / TW) * PPL;
    }
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
      const int x = tx * TW + lx, y = ty * TH + ly0 + q;
      const bool in = x < cam.width && y < cam.height;
      loc[q] = (ly0 + q) * TW + lx;
      pix[q] = in ? (int)(y * cam.width + x) : -1;
      pxc[q] = (float)x + 0.5f;
      pyc[q] = (float)y + 0.5f;
      const float cxn = (pxc[q] - cam.cx) / cam.fx;
      const float cyn = (pyc[q] - cam.cy) / cam.fy;
      const float Dx = cam.Rinv_f[0] * cxn + cam.Rinv_f[1] * cyn + cam.Rinv_f[2];
      const float Dy = cam.Rinv_f[3] * cxn + cam.Rinv_f[4] * cyn + cam.Rinv_f[5];
      const float Dz = cam.Rinv_f[6] * cxn + cam.Rinv_f[7] * cyn + cam.Rinv_f[8];
      L[q] = sqrtf(Dx * Dx + Dy * Dy + Dz * Dz);
    }
  }
};

// LDS stage of one batch: records and tables.
template <int N, int B>
struct Stage {
  static constexpr int NB = B;
  static constexpr int TS = 5 * N + 4;
  static constexpr int F = 6 + TS / 4;  // float4 per instance
  float4 rec[B][6];
  float4 tab[B][TS / 4];
  int4 rect[B];  // the primitive's inclusive pixel rectangle in this view
  uint32_t id[B];
};

// Per-ray colour network of a batch (colour mode 4, width 16, CD hidden
// layers): each instance's table row and its view's first-layer bias.
template <int CD, int B>
struct ColourStage {
  static constexpr int T4 = RayColourLayout<16, CD>::CTS / 4;
  float4 t[B][T4];
  float4 b[B][4];
};

// Stages one batch: instance ids and rectangles, records and tables (and,
// with a colour stage, the colour tables and biases), gathered by primitive
// id as float4.  The
// threads that gather read the id from global memory themselves, so one
// barrier (at the end) suffices.  The caller's previous barrier (the end of
// the previous batch, or the work-queue fetch) guarantees nobody still
// reads the stage.
template <int N, int NT, int B, int CD = 0>
__device__ __forceinline__ void stage_batch(Stage<N, B>& S, const RasterArgs& a, int v, uint32_t b0, int nb,
                                            ColourStage<(CD > 0 ? CD : 1), B>* cs = nullptr) {
  const int64_t vbase = (int64_t)v * a.P;
  for (int t = threadIdx.x; t < nb; t += NT) {
    const uint32_t p = a.values[b0 + t];
    S.id[t] = p;
    S.rect[t] = reinterpret_cast<const int4*>(a.rects)[vbase + p];
  }
  const float4* rec4 = reinterpret_cast<const float4*>(a.records);
  const float4* tab4 = reinterpret_cast<const float4*>(a.table);
  constexpr int F = Stage<N, B>::F;
  constexpr int T4 = Stage<N, B>::TS / 4;
  for (int idx = threadIdx.x; idx < nb * F; idx += NT) {
    const int j = idx / F, c = idx - j * F;
    const uint32_t p = a.values[b0 + j];
    if (c < 6)
      S.rec[j][c] = rec4[(vbase + p) * 6 + c];
    else
      S.tab[j][c - 6] = tab4[(int64_t)p * T4 + (c - 6)];
  }
  if constexpr (CD > 0) {
    constexpr int C4 = ColourStage<CD, B>::T4;
    const float4* ct4 = reinterpret_cast<const float4*>(a.ctab);
    const float4* cb4 = reinterpret_cast<const float4*>(a.cbias);
    for (int idx = threadIdx.x; idx < nb * (C4 + 4); idx += NT) {
      const int j = idx / (C4 + 4), c = idx - j * (C4 + 4);
      const uint32_t p = a.values[b0 + j];
      if (c < C4)
        cs->t[j][c] = ct4[(int64_t)p * C4 + c];
      else
        cs->b[j][c - C4] = cb4[(vbase + p) * 4 + (c - C4)];
    }
  }
  __syncthreads();
}

// The per-ray colour network on one pair: the entry point u (unit-sphere
// frame) and the ray direction n = d'/L give the first layer, ReLU hidden
// layers, sigmoid output (kept with the activations for the adjoint).
template <int CD>
struct RayAct {
  float h1[16];
  float h2[CD == 2 ? 16 : 1];
  float sg[3];
};

// 0, as an opaque value computed after x: weight reads indexed with it
// cannot be issued before x exists, which keeps the compiler from hoisting a
// whole network's LDS reads ahead of its arithmetic (and holding them in
// registers).
__device__ __forceinline__ int zero_after(float x) {
  int z = 0;
  asm volatile("" : "+v"(z) : "v"(x));
  return z;
}

template <int CD>
__device__ __forceinline__ void ray_net(const float* ct, const float* cb, float u0, float u1, float u2, float n0,
                                        float n1, float n2, RayAct<CD>& r) {
  using Lt = RayColourLayout<16, CD>;
  int z = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const float* w = ct + z;
    float h = cb[z + k];
    h = __builtin_fmaf(w[Lt::AU + 3 * k + 0], u0, h);
    h = __builtin_fmaf(w[Lt::AU + 3 * k + 1], u1, h);
    h = __builtin_fmaf(w[Lt::AU + 3 * k + 2], u2, h);
    h = __builtin_fmaf(w[Lt::AD + 3 * k + 0], n0, h);
    h = __builtin_fmaf(w[Lt::AD + 3 * k + 1], n1, h);
    h = __builtin_fmaf(w[Lt::AD + 3 * k + 2], n2, h);
    r.h1[k] = fmaxf(h, 0.f);
    if (k & 1) z = zero_after(h);  // the next two units' reads wait for these
  }
  if constexpr (CD == 2) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      float h = ct[Lt::BH + k];
#pragma unroll
      for (int i = 0; i < 16; ++i) h = __builtin_fmaf(ct[Lt::WH + 16 * k + i], r.h1[i], h);
      r.h2[k] = fmaxf(h, 0.f);
      asm volatile("" ::: "memory");  // one row of Wh in registers at a time
    }
  }
  const float* hl = CD == 2 ? r.h2 : r.h1;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float* w = ct + z;
    float o = w[Lt::BO + c];
#pragma unroll
    for (int k = 0; k < 16; ++k) o = __builtin_fmaf(w[Lt::WO + 16 * c + k], hl[k], o);
    r.sg[c] = fast_rcp(1.f + exp2_fast(-o * kLog2e));
    z = zero_after(o);
  }
}

// The colour alone (the forward and the backward's pixel phase): with one
// hidden layer each unit goes straight into the three output sums, so no
// activation is kept.  The unit loop is unrolled by two only: fully
// unrolled, the compiler issues all 160 weight reads (LDS broadcasts) ahead
// of the arithmetic and holds them in registers, which halves the waves a
// SIMD can keep.
template <int CD>
__device__ __forceinline__ void ray_colour(const float* ct, const float* cb, float u0, float u1, float u2, float n0,
                                           float n1, float n2, float* sg) {
  if constexpr (CD == 1) {
    using Lt = RayColourLayout<16, 1>;
    float o0 = ct[Lt::BO + 0], o1 = ct[Lt::BO + 1], o2 = ct[Lt::BO + 2];
#pragma unroll 2
    for (int k = 0; k < 16; ++k) {
      float h = cb[k];
      h = __builtin_fmaf(ct[Lt::AU + 3 * k + 0], u0, h);
      h = __builtin_fmaf(ct[Lt::AU + 3 * k + 1], u1, h);
      h = __builtin_fmaf(ct[Lt::AU + 3 * k + 2], u2, h);
      h = __builtin_fmaf(ct[Lt::AD + 3 * k + 0], n0, h);
      h = __builtin_fmaf(ct[Lt::AD + 3 * k + 1], n1, h);
      h = __builtin_fmaf(ct[Lt::AD + 3 * k + 2], n2, h);
      h = fmaxf(h, 0.f);
      o0 = __builtin_fmaf(ct[Lt::WO + k], h, o0);
      o1 = __builtin_fmaf(ct[Lt::WO + 16 + k], h, o1);
      o2 = __builtin_fmaf(ct[Lt::WO + 32 + k], h, o2);
    }
    sg[0] = fast_rcp(1.f + exp2_fast(-o0 * kLog2e));
    sg[1] = fast_rcp(1.f + exp2_fast(-o1 * kLog2e));
    sg[2] = fast_rcp(1.f + exp2_fast(-o2 * kLog2e));
  } else {
    RayAct<CD> r;
    ray_net<CD>(ct, cb, u0, u1, u2, n0, n1, n2, r);
    sg[0] = r.sg[0];
    sg[1] = r.sg[1];
    sg[2] = r.sg[2];
  }
}

// geometry of one (pixel, primitive) pair from a staged record
struct PairGeom {
  float dx, dy;
  float d0, d1, d2, m0, m1, m2;
  float A, rA, sq, H;
  float p0, p1, p2, e0, e1, e2;
};

// dqg: the float64 coefficients of the discriminant as a quadratic in the
// pixel offset from the record's reference pixel (in global memory; the
// pointer is the same for the whole wave).  The float32 discriminant A - M
// is within band/64 of the exact one (r5.w, from a bound on its rounding
// errors over the rectangle), so outside the band its sign decides a hit;
// inside it the float64 form, evaluated at the exact offset (the difference
// of two floats is exact in float64), decides the hit and gives the value.
// The oracle decides with its own float64 discriminant, so the hit pairs of
// both sides are the same pairs (up to ties within float64 rounding).  The
// forward and the pixel phase of the backward call this with the same band,
// so they agree on every hit and every value; the gradient phase widens the
// band to 1% of A (WIDE), where the float32 value has too few correct digits
// for the 1/sqrt(disc) factor of the geometry gradient.
// d', m' and A = |d'|^2 at a pixel centre from a staged record
__device__ __forceinline__ void pair_dm(const float4& r0, const float4& r1, const float4& r2, const float4& r3,
                                        const float4& r4, const float4& r5, float px, float py, PairGeom& g) {
  g.dx = px - r0.w;
  g.dy = py - r1.w;
  g.d0 = __builtin_fmaf(r2.x, g.dy, __builtin_fmaf(r1.x, g.dx, r0.x));
  g.d1 = __builtin_fmaf(r2.y, g.dy, __builtin_fmaf(r1.y, g.dx, r0.y));
  g.d2 = __builtin_fmaf(r2.z, g.dy, __builtin_fmaf(r1.z, g.dx, r0.z));
  g.m0 = __builtin_fmaf(r5.x, g.dy, __builtin_fmaf(r4.x, g.dx, r3.x));
  g.m1 = __builtin_fmaf(r5.y, g.dy, __builtin_fmaf(r4.y, g.dx, r3.y));
  g.m2 = __builtin_fmaf(r5.z, g.dy, __builtin_fmaf(r4.z, g.dx, r3.z));
  g.A = __builtin_fmaf(g.d2, g.d2, __builtin_fmaf(g.d1, g.d1, g.d0 * g.d0));
}

template <bool WIDE = false>
__device__ __forceinline__ bool pair_geom(const float4& r0, const float4& r1, const float4& r2, const float4& r3,
                                          const float4& r4, const float4& r5, float px, float py, PairGeom& g,
                                          const double* dqg) {
  pair_dm(r0, r1, r2, r3, r4, r5, px, py, g);
  const float M = __builtin_fmaf(g.m2, g.m2, __builtin_fmaf(g.m1, g.m1, g.m0 * g.m0));
  float disc = g.A - M;
  bool hit = disc > 0.f;
  const float band = WIDE ? fmaxf(r5.w, 0.01f * g.A) : r5.w;
  if (fabsf(disc) < band) {
    const double x = (double)px - (double)r0.w, y = (double)py - (double)r1.w;
    const double dd = dqg[0] + x * (dqg[1] + dqg[3] * x + dqg[4] * y) + y * (dqg[2] + dqg[5] * y);
    hit = dd > 0.0;
    disc = (float)dd;
  }
  // every field stays finite for a miss (H = 0, e' = 0), so loops over the
  // hidden units can run without per-pixel branches and be masked afterwards
  g.rA = fast_rcp(g.A);
  g.sq = fast_sqrt(hit ? fmaxf(disc, 0.f) : 0.f);
  g.H = g.sq * g.rA;
  g.p0 = (g.d1 * g.m2 - g.d2 * g.m1) * g.rA;
  g.p1 = (g.d2 * g.m0 - g.d0 * g.m2) * g.rA;
  g.p2 = (g.d0 * g.m1 - g.d1 * g.m0) * g.rA;
  g.e0 = g.d0 * g.H;
  g.e1 = g.d1 * g.H;
  g.e2 = g.d2 * g.H;
  return hit;
}

// the float64 discriminant coefficients of staged instance j (the address
// is the same for the whole wave, so the loads are scalar)
template <int N, int B>
__device__ __forceinline__ const double* disc_coef_of(const Stage<N, B>& S, const RasterArgs& a, int v, int j) {
  const uint32_t p = __builtin_amdgcn_readfirstlane(S.id[j]);
  return a.disc_coef + ((int64_t)v * a.P + p) * 6;
}

__device__ __forceinline__ float alpha_of(float ahat, float alpha_max) {
  const float al = ahat > 0.f ? 1.0f - exp2_fast(-ahat * kLog2e) : 0.f;
  return fminf(al, alpha_max);
}

// adds the wave's total of v to *slot (one atomic per wave)
__device__ __forceinline__ void count_tile_pairs(uint32_t* slot, uint32_t v) {
  for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(slot, v);
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
// CD > 0: the per-ray colour network of colour mode 4 (depth CD, width 16)
// colours each pair; otherwise the pair takes its record's colour.
template <int N, int TW, int TH, int PPL, bool PERSIST, bool COUNT, int CD = 0>
__global__ void __launch_bounds__(TW * TH / PPL) render_fwd_kernel(RasterArgs a) {
  constexpr int NT = TW * TH / PPL;
  constexpr int FB = fwd_batch<N, CD>();
  __shared__ Stage<N, FB> S;
  __shared__ ColourStage<(CD > 0 ? CD : 1), (CD > 0 ? FB : 1)> CS;
  __shared__ int s_item;
  unsigned long long npairs = 0, nlive = 0;
  int item = blockIdx.x;
  while (true) {
    if (PERSIST) {
      if (threadIdx.x == 0) s_item = (int)atomicAdd(&a.counters[CNT_QUEUE_FWD], 1ull);
      __syncthreads();
      item = s_item;
      __syncthreads();
    }
    if (item >= a.total_tiles) break;
    // persistent launches take the tiles in the order of tile_order (most
    // instances first), so the heaviest tiles do not form the tail
    const int tile = (PERSIST && a.tile_order) ? (int)a.tile_order[item] : item;
    const int v = view_of_tile(a.cams, a.V, tile);
    const CamDev& cam = a.cams[v];
    const int local = tile - cam.tile_base;
    const int ty = local / cam.ntx, tx = local - ty * cam.ntx;
    PixelBlock<TW, TH, PPL> pb;
    pb.init(cam, tx, ty);
    float T[PPL], C0[PPL], C1[PPL], C2[PPL];
    bool done[PPL];
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
      T[q] = 1.f;
      C0[q] = C1[q] = C2[q] = 0.f;
      done[q] = pb.pix[q] < 0;
    }
    uint32_t tpairs = 0;  // this thread's hit pairs in this tile (COUNT)
    const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
    for (uint32_t b0 = start; b0 < end; b0 += FB) {
      const int nb = (int)min((uint32_t)FB, end - b0);
      if constexpr (CD > 0)
        stage_batch<N, NT, FB, CD>(S, a, v, b0, nb, &CS);
      else
        stage_batch<N, NT, FB>(S, a, v, b0, nb);
#pragma unroll 1
      for (int j = 0; j < nb; ++j) {
        const int4 rc = S.rect[j];
        if (rc.y < pb.wx0 || rc.x > pb.wx1 || rc.w < pb.wy0 || rc.z > pb.wy1) continue;  // wave-uniform
        const float4 r0 = S.rec[j][0], r1 = S.rec[j][1], r2 = S.rec[j][2];
        const float4 r3 = S.rec[j][3], r4 = S.rec[j][4], r5 = S.rec[j][5];
        const double* dqj = disc_coef_of(S, a, v, j);
        PairGeom g[PPL];
        bool hit[PPL];
        bool any = false;
        float Q[PPL];
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
          // geometry for every lane (finite for misses), so the unit loops can run unmasked
          const bool gh = pair_geom(r0, r1, r2, r3, r4, r5, pb.pxc[q], pb.pyc[q], g[q], dqj);
          hit[q] = !done[q] && gh;
          any |= hit[q];
          Q[q] = 0.f;
          if (COUNT) tpairs += hit[q] ? 1u : 0u;
        }
        if (__ballot(any) == 0) continue;  // wave-uniform skip
        const float* tabf = reinterpret_cast<const float*>(S.tab[j]);
        // all lanes run the unit loop; misses are masked after it
#pragma unroll 4
        for (int k = 0; k < N; ++k) {
          const float4 w = S.tab[j][k];
          const float w2 = tabf[4 * N + k];
#pragma unroll
          for (int q = 0; q < PPL; ++q) {
            const float ph = __builtin_fmaf(w.x, g[q].p0, __builtin_fmaf(w.y, g[q].p1, __builtin_fmaf(w.z, g[q].p2, w.w)));
            const float hv = __builtin_fmaf(w.x, g[q].e0, __builtin_fmaf(w.y, g[q].e1, w.z * g[q].e2));
            const float c = cos_rev(ph);
            const float sn = sinc_rev(sin_rev(hv), hv);
            Q[q] = __builtin_fmaf(w2 * c, sn, Q[q]);
          }
        }
        const float b2 = tabf[5 * N];
        float ahat[PPL];
#pragma unroll
        for (int q = 0; q < PPL; ++q) ahat[q] = 2.f * pb.L[q] * g[q].H * (Q[q] + b2);
        if (a.ahat_cache && (int64_t)(b0 + j) < a.cache_instances) {  // every lane of an evaluated wave stores (misses store 0)
          float* cp = a.ahat_cache + (int64_t)(b0 + j) * (TW * TH);
#pragma unroll
          for (int q = 0; q < PPL; ++q) cp[pb.loc[q]] = ahat[q];
        }
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
          // the pair's colour: the record's, or c_dc + the per-ray network at
          // the entry point u = p' - e' with the direction d' / L
          float c0 = r2.w, c1 = r3.w, c2 = r4.w;
          if constexpr (CD > 0) {
            float sg[3];
            const float iL = fast_rcp(pb.L[q]);
            ray_colour<CD>(reinterpret_cast<const float*>(CS.t[j]), reinterpret_cast<const float*>(CS.b[j]),
                           g[q].p0 - g[q].e0, g[q].p1 - g[q].e1, g[q].p2 - g[q].e2, g[q].d0 * iL, g[q].d1 * iL,
                           g[q].d2 * iL, sg);
            c0 += sg[0];
            c1 += sg[1];
            c2 += sg[2];
          }
          // without branches: a lane that does not blend this pair (a miss,
          // a terminated pixel, an alpha_min skip) takes alpha = 0, which
          // leaves its colour and T exactly as they were
          const float al0 = alpha_of(ahat[q], a.alpha_max);
          if (COUNT) nlive += (hit[q] && ahat[q] > 0.f && al0 < a.alpha_max) ? 1 : 0;
          const bool blend = hit[q] && !(a.alpha_min > 0.f && al0 < a.alpha_min);
          const float al = blend ? al0 : 0.f;
          const float w = al * T[q];
          C0[q] = __builtin_fmaf(c0, w, C0[q]);
          C1[q] = __builtin_fmaf(c1, w, C1[q]);
          C2[q] = __builtin_fmaf(c2, w, C2[q]);
          T[q] = T[q] * (1.f - al);
          done[q] = done[q] || T[q] < a.t_eps;
        }
      }
      bool mine = true;
#pragma unroll
      for (int q = 0; q < PPL; ++q) mine = mine && done[q];
      if (__syncthreads_and(mine)) break;
    }
    if (COUNT) {
      npairs += tpairs;
      count_tile_pairs(a.tile_pairs + tile, tpairs);
    }
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
      if (pb.pix[q] >= 0) {
        const int64_t px = cam.pix_base + pb.pix[q];
        a.images[3 * px + 0] = C0[q] + T[q] * a.bg0;
        a.images[3 * px + 1] = C1[q] + T[q] * a.bg1;
        a.images[3 * px + 2] = C2[q] + T[q] * a.bg2;
        a.final_T[px] = T[q];
      }
    }
    if (!PERSIST) break;
  }
  if (COUNT) {
    // one atomic per wave
    unsigned long long tot = npairs, live = nlive;
    for (int o = 1; o < 64; o <<= 1) {
      tot += __shfl_xor(tot, o);
      live += __shfl_xor(live, o);
    }
    if ((threadIdx.x & 63) == 0) {
      atomicAdd(&a.counters[CNT_HIT_PAIRS], tot);
      atomicAdd(&a.counters[CNT_LIVE_PAIRS], live);
    }
  }
}

// ---------------------------------------------------------------------------
// forward of Gaussian splats (the 3DGS kernel of the paper's comparison,
// App. A): per pixel inside the primitive's rectangle,
//   alpha = min(alpha_max, opacity 2^(ka dx^2 + kb dx dy + kc dy^2)),
// blended like the neural primitives.  A batch is one instance per thread
// (up to the workgroup size), staged as two float4, the blue channel and
// the rectangle.
// ---------------------------------------------------------------------------
template <int NT>
struct GaussStage {
  float4 g0[NT];  // u, v, ka, red
  float4 g1[NT];  // kb, kc, opacity, green
  float cb[NT];   // blue
  int4 rect[NT];
};

template <int TW, int TH, int PPL, bool PERSIST, bool COUNT>
__global__ void __launch_bounds__(TW * TH / PPL) render_fwd_gauss_kernel(RasterArgs a) {
  constexpr int NT = TW * TH / PPL;
  __shared__ GaussStage<NT> S;
  __shared__ int s_item;
  unsigned long long npairs = 0, nlive = 0;
  int item = blockIdx.x;
  while (true) {
    if (PERSIST) {
      if (threadIdx.x == 0) s_item = (int)atomicAdd(&a.counters[CNT_QUEUE_FWD], 1ull);
      __syncthreads();
      item = s_item;
      __syncthreads();
    }
    if (item >= a.total_tiles) break;
    // persistent launches take the tiles in the order of tile_order (most
    // instances first), so the heaviest tiles do not form the tail
    const int tile = (PERSIST && a.tile_order) ? (int)a.tile_order[item] : item;
    const int v = view_of_tile(a.cams, a.V, tile);
    const CamDev& cam = a.cams[v];
    const int local = tile - cam.tile_base;
    const int ty = local / cam.ntx, tx = local - ty * cam.ntx;
    PixelBlock<TW, TH, PPL> pb;
    pb.init(cam, tx, ty);
    int px[PPL], py[PPL];
    float T[PPL], C0[PPL], C1[PPL], C2[PPL];
    bool done[PPL];
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
      px[q] = (int)pb.pxc[q];
      py[q] = (int)pb.pyc[q];
      T[q] = 1.f;
      C0[q] = C1[q] = C2[q] = 0.f;
      done[q] = pb.pix[q] < 0;
    }
    const int64_t vbase = (int64_t)v * a.P;
    const float4* rec4 = reinterpret_cast<const float4*>(a.records);
    uint32_t tpairs = 0;  // this thread's hit pairs in this tile (COUNT)
    const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
    for (uint32_t b0 = start; b0 < end; b0 += NT) {
      const int nb = (int)min((uint32_t)NT, end - b0);
      if ((int)threadIdx.x < nb) {
        const int64_t r = vbase + a.values[b0 + threadIdx.x];
        S.rect[threadIdx.x] = reinterpret_cast<const int4*>(a.rects)[r];
        S.g0[threadIdx.x] = rec4[r * 6 + 2];
        S.g1[threadIdx.x] = rec4[r * 6 + 3];
        S.cb[threadIdx.x] = a.records[r * kRecFloats + 19];
      }
      __syncthreads();
#pragma unroll 4
      for (int j = 0; j < nb; ++j) {
        const int4 rc = S.rect[j];
        if (rc.y < pb.wx0 || rc.x > pb.wx1 || rc.w < pb.wy0 || rc.z > pb.wy1) continue;  // wave-uniform
        const float4 g0 = S.g0[j], g1 = S.g1[j];
        const float blue = S.cb[j];
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
          const bool hit = !done[q] && px[q] >= rc.x && px[q] <= rc.y && py[q] >= rc.z && py[q] <= rc.w;
          if (COUNT) tpairs += hit ? 1u : 0u;
          const float dx = pb.pxc[q] - g0.x, dy = pb.pyc[q] - g0.y;
          // log2 of the Gaussian factor; <= 0 for the positive definite conic
          const float pw = fminf(__builtin_fmaf(dx, __builtin_fmaf(g1.x, dy, g0.z * dx), g1.y * dy * dy), 0.f);
          const float al = fminf(g1.z * exp2_fast(pw), a.alpha_max);
          if (hit && !(a.alpha_min > 0.f && al < a.alpha_min)) {
            if (COUNT) nlive += 1;
            const float w = al * T[q];
            C0[q] = __builtin_fmaf(g0.w, w, C0[q]);
            C1[q] = __builtin_fmaf(g1.w, w, C1[q]);
            C2[q] = __builtin_fmaf(blue, w, C2[q]);
            T[q] = T[q] * (1.f - al);
            if (T[q] < a.t_eps) done[q] = true;
          }
        }
      }
      bool mine = true;
#pragma unroll
      for (int q = 0; q < PPL; ++q) mine = mine && done[q];
      if (__syncthreads_and(mine)) break;
    }
    if (COUNT) {
      npairs += tpairs;
      count_tile_pairs(a.tile_pairs + tile, tpairs);
    }
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
      if (pb.pix[q] >= 0) {
        const int64_t pxi = cam.pix_base + pb.pix[q];
        a.images[3 * pxi + 0] = C0[q] + T[q] * a.bg0;
        a.images[3 * pxi + 1] = C1[q] + T[q] * a.bg1;
        a.images[3 * pxi + 2] = C2[q] + T[q] * a.bg2;
        a.final_T[pxi] = T[q];
      }
    }
    if (!PERSIST) break;
  }
  if (COUNT) {
    unsigned long long tot = npairs, live = nlive;
    for (int o = 1; o < 64; o <<= 1) {
      tot += __shfl_xor(tot, o);
      live += __shfl_xor(live, o);
    }
    if ((threadIdx.x & 63) == 0) {
      atomicAdd(&a.counters[CNT_HIT_PAIRS], tot);
      atomicAdd(&a.counters[CNT_LIVE_PAIRS], live);
    }
  }
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
// sum over each row of 16 lanes; every lane of the row ends with its row's sum
__device__ __forceinline__ float dpp_row_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));  // row_half_mirror
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false));  // row_mirror
  return v;
}

// adds the wave's sum of v into an LDS accumulator: row sums, then one LDS
// atomic per row (4 lanes)
__device__ __forceinline__ void wave_accumulate(float* slot, float v, int lane) {
  v = dpp_row_sum(v);
  if ((lane & 15) == 0) atomicAdd(slot, v);
}

// five sums at once (interleaved, so the DPP steps of one value fill the
// hazard slots of the others): a[0..3] += (x, y, z, w), b[0] += u
__device__ __forceinline__ void wave_accumulate5(float* a, float* b, float x, float y, float z, float w, float u,
                                                 int lane) {
#define SNP_DPP_STEP(CTRL)                                                                          \
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false)); \
  y += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(y), CTRL, 0xF, 0xF, false)); \
  z += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(z), CTRL, 0xF, 0xF, false)); \
  w += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(w), CTRL, 0xF, 0xF, false)); \
  u += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(u), CTRL, 0xF, 0xF, false));
  SNP_DPP_STEP(0xB1)
  SNP_DPP_STEP(0x4E)
  SNP_DPP_STEP(0x141)
  SNP_DPP_STEP(0x140)
#undef SNP_DPP_STEP
  if ((lane & 15) == 0) {
    atomicAdd(a + 0, x);
    atomicAdd(a + 1, y);
    atomicAdd(a + 2, z);
    atomicAdd(a + 3, w);
    atomicAdd(b, u);
  }
}

// Transposed butterfly over the 16 lanes of a row.  One level combines two
// registers a, b across partner lanes: a lane whose selector bit is set keeps
// b and sends a, its partner keeps a and sends b, and each adds what it
// receives, so the pair of lanes ends with the pair sum of a in one lane and
// of b in the other.  Four levels with partners lane^7 (row_half_mirror),
// lane^1, lane^2 and lane^8 (row_ror:8) and selector bits 2, 0, 1, 3 reduce
// 16 registers to one in which row lane r holds the row sum of value
// 8 b3 + 4 b1 + 2 b0 + b2 (b = the bits of r): 45 VALU operations for 16
// sums, against 64 and 16 LDS atomics for one plain butterfly per value.
constexpr int kDppXor1 = 0xB1;        // quad_perm 1,0,3,2
constexpr int kDppXor2 = 0x4E;        // quad_perm 2,3,0,1
constexpr int kDppHalfMirror = 0x141; // row_half_mirror: lane ^ 7 within 8
constexpr int kDppRor8 = 0x128;       // row_ror:8: lane ^ 8 within the row

template <int CTRL>
__device__ __forceinline__ float dpp_from_partner(float v) {
  // every lane has a source lane in the patterns used here, so bound_ctrl
  // changes nothing but lets the move fold into the consuming add
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

template <int CTRL>
__device__ __forceinline__ float tb_level(float a, float b, bool sel) {
  const float keep = sel ? b : a, send = sel ? a : b;
  return keep + dpp_from_partner<CTRL>(send);
}

// plain butterfly level (one value): both partners end with the pair sum
template <int CTRL>
__device__ __forceinline__ float nb_level(float a) {
  return a + dpp_from_partner<CTRL>(a);
}

// Sums across the four rows of 16 lanes (v_permlane32_swap exchanges the
// upper half of its first operand with the lower half of its second,
// v_permlane16_swap the odd rows of the first with the even rows of the
// second).  cross_rows_sum: every row ends with the sum of the four rows.
__device__ __forceinline__ float cross_rows_sum(float x) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  const float s = __uint_as_float(r[0]) + __uint_as_float(r[1]);  // rows: x0+x2, x1+x3, x0+x2, x1+x3
  const auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(s), __float_as_uint(s), false, false);
  return __uint_as_float(q[0]) + __uint_as_float(q[1]);
}

// Two registers of row partials: rows 0 and 1 end with the four-row sums
// of a, rows 2 and 3 with those of b.
__device__ __forceinline__ float cross_rows_pair(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  const float w = __uint_as_float(r[0]) + __uint_as_float(r[1]);  // rows: a0+a2, a1+a3, b0+b2, b1+b3
  const auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(w), __float_as_uint(w), false, false);
  return __uint_as_float(q[0]) + __uint_as_float(q[1]);
}

// d/dh of sin(2 pi h)/h near h = 0 is -(2 pi)^3 h / 3 + (2 pi)^5 h^3 / 30
// (the next term, (2 pi)^7 h^5 / 840, is below float rounding for
// |h| < 0.02); these are its coefficients divided by -2 pi
constexpr float kDsnC1n = (kTwoPi * kTwoPi) / 3.0f;
constexpr float kDsnC3n = -(kTwoPi * kTwoPi * kTwoPi * kTwoPi) / 30.0f;

// Sum over the wave of 16 values: lane l < 16 ends with the sum of value
// 8 b3 + 4 b1 + 2 b0 + b2 (b = the bits of l).
__device__ __forceinline__ float wave_sum16(const float* v, bool sel1, bool sel2, bool sel3, bool sel4) {
  float x4[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    x4[q] = tb_level<kDppXor1>(tb_level<kDppHalfMirror>(v[4 * q], v[4 * q + 1], sel1),
                               tb_level<kDppHalfMirror>(v[4 * q + 2], v[4 * q + 3], sel1), sel2);
  return cross_rows_sum(tb_level<kDppRor8>(tb_level<kDppXor2>(x4[0], x4[1], sel3),
                                           tb_level<kDppXor2>(x4[2], x4[3], sel3), sel4));
}

// Adjoint of the per-ray colour network on the wave's 64 pairs (every lane
// takes part; a lane without a pair passes gc = 0).  gc: d loss / d colour
// of the lane's pair.  The weight gradients summed over the wave go to the
// primitive's table gradient gt and the (view, primitive) bias gradient gb
// (global), the offset c_dc's to acc_col (LDS); returns d loss / d u and
// d loss / d n of the lane's pair.
template <int CD>
__device__ __forceinline__ void ray_net_adjoint(const float* ct, const float* cb, float u0, float u1, float u2,
                                                float n0, float n1, float n2, float gc0, float gc1, float gc2,
                                                float* gt, float* gb, float* acc_col, int lane, int idx16,
                                                bool sel1, bool sel2, bool sel3, bool sel4, float* gu, float* gn) {
  using Lt = RayColourLayout<16, CD>;
  RayAct<CD> ra;
  ray_net<CD>(ct, cb, u0, u1, u2, n0, n1, n2, ra);
  const float go[3] = {gc0 * ra.sg[0] * (1.f - ra.sg[0]), gc1 * ra.sg[1] * (1.f - ra.sg[1]),
                       gc2 * ra.sg[2] * (1.f - ra.sg[2])};
  auto flush16 = [&](float* base, const float* v16) {
    const float z = wave_sum16(v16, sel1, sel2, sel3, sel4);
    if (lane < 16 && z != 0.f) atomic_add_f32(base + idx16, z);
    asm volatile("" ::: "memory");  // one block of 16 sums in registers at a time
  };
  const float* hl = CD == 2 ? ra.h2 : ra.h1;
  float v[16];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = go[c] * hl[k];
    flush16(gt + Lt::WO + 16 * c, v);
  }
  {
    // output bias and the colour offset
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = 0.f;
    v[0] = go[0];
    v[1] = go[1];
    v[2] = go[2];
    v[3] = gc0;
    v[4] = gc1;
    v[5] = gc2;
    const float z = wave_sum16(v, sel1, sel2, sel3, sel4);
    if (lane < 16 && z != 0.f) {
      if (idx16 < 3)
        atomic_add_f32(gt + Lt::BO + idx16, z);
      else if (idx16 < 6)
        atomicAdd(acc_col + idx16 - 3, z);
    }
  }
  // d loss / d pre-activation of the last hidden layer
  float gh[16];
  int z = zero_after(go[2]);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const float* w = ct + z;
    const float t = go[0] * w[Lt::WO + k] + go[1] * w[Lt::WO + 16 + k] + go[2] * w[Lt::WO + 32 + k];
    gh[k] = hl[k] > 0.f ? t : 0.f;
    if ((k & 3) == 3) z = zero_after(t);
  }
  if constexpr (CD == 2) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = gh[r] * ra.h1[i];
      flush16(gt + Lt::WH + 16 * r, v);
    }
    flush16(gt + Lt::BH, gh);
    float g1[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      float t = 0.f;
#pragma unroll
      for (int r = 0; r < 16; ++r) t = __builtin_fmaf(ct[Lt::WH + 16 * r + i], gh[r], t);
      g1[i] = ra.h1[i] > 0.f ? t : 0.f;
      asm volatile("" ::: "memory");
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) gh[i] = g1[i];
  }
  // first layer: Au (k * 3 + j), Ad, the bias
  const float uu[3] = {u0, u1, u2}, nn[3] = {n0, n1, n2};
#pragma unroll
  for (int b = 0; b < 3; ++b) {
#pragma unroll
    for (int t = 0; t < 16; ++t) v[t] = gh[(16 * b + t) / 3] * uu[(16 * b + t) % 3];
    flush16(gt + Lt::AU + 16 * b, v);
  }
#pragma unroll
  for (int b = 0; b < 3; ++b) {
#pragma unroll
    for (int t = 0; t < 16; ++t) v[t] = gh[(16 * b + t) / 3] * nn[(16 * b + t) % 3];
    flush16(gt + Lt::AD + 16 * b, v);
  }
  flush16(gb, gh);
  z = zero_after(gh[15]);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const float* w = ct + z;
    float tu = 0.f, tn = 0.f;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      tu = __builtin_fmaf(w[Lt::AU + 3 * k + j], gh[k], tu);
      tn = __builtin_fmaf(w[Lt::AD + 3 * k + j], gh[k], tn);
    }
    gu[j] = tu;
    gn[j] = tn;
    z = zero_after(tn);
  }
}

// Length of the un-normalised camera ray R^-1 ((x+1/2-cx)/fx, (y+1/2-cy)/fy, 1).
__device__ __forceinline__ float ray_length(const CamDev& cam, float pxc, float pyc) {
  const float cxn = (pxc - cam.cx) / cam.fx;
  const float cyn = (pyc - cam.cy) / cam.fy;
  const float Dx = cam.Rinv_f[0] * cxn + cam.Rinv_f[1] * cyn + cam.Rinv_f[2];
  const float Dy = cam.Rinv_f[3] * cxn + cam.Rinv_f[4] * cyn + cam.Rinv_f[5];
  const float Dz = cam.Rinv_f[6] * cxn + cam.Rinv_f[7] * cyn + cam.Rinv_f[8];
  return sqrtf(Dx * Dx + Dy * Dy + Dz * Dz);
}

// The backward works on batches of NB instances of a tile in two phases.
//
// Phase 1 (one pixel per thread, the instances in depth order): the same
// arithmetic as the forward gives alpha, T and the accumulated colour; the
// colour gradient is summed here; every pair whose integral is positive and
// unclamped ("live", it carries gradient) is appended to the instance's list
// in LDS with its pixel, d loss / d Q and d loss / d H.
//
// Phase 2 (one live pair per lane): the waves take chunks of 64 list entries
// (instance by instance, round robin over the waves), recompute the pair's
// geometry -- with the float64 discriminant near the silhouette -- and the
// per-unit terms, and sum the gradients of the table entries and of the
// record coefficients over the wave into LDS accumulators, flushed to HBM
// once per batch.  Every lane of phase 2 carries gradient, and each wave
// reduction covers 64 live pairs.
//
// With the per-ray colour network (CD > 0, colour mode 4) phase 1 evaluates
// each pair's colour, lists every pair that blends (alpha > 0) with its
// weight alpha T, and phase 2 adds the network's adjoint: the weight
// gradients summed over the 64 pairs into the per-primitive table gradient
// (and the per-(view, primitive) bias gradient), the colour offset into the
// record gradient, and the entry point's and direction's gradients into the
// geometry chain.
template <int N, int TW, int TH, int NB, bool PERSIST, int CD = 0>
__global__ void __launch_bounds__(TW * TH) __attribute__((amdgpu_waves_per_eu(CD > 0 ? 4 : 5)))
render_bwd_kernel(RasterArgs a) {
  constexpr int NT = TW * TH;
  constexpr int NW = NT / 64;
  constexpr int TS = 5 * N + 4;
  constexpr int ACC = TS + kGViewFloats;  // per instance: table grads, then record grads
  __shared__ Stage<N, NB> S;
  __shared__ float s_acc[NB][ACC];
  __shared__ uint32_t s_cnt[NB][NW];  // live pairs per (instance, wave)
  // the pair's pixel within the tile (one byte where it fits; only the
  // per-ray colour kernels need the LDS it saves)
  using PixIndex = std::conditional_t<(CD > 0 && NT <= 256), uint8_t, uint16_t>;
  __shared__ PixIndex s_pix[NB][NT];
  __shared__ float s_wq[NB][NT];
  __shared__ float s_gh[NB][NT];
  __shared__ ColourStage<(CD > 0 ? CD : 1), (CD > 0 ? NB : 1)> CS;
  __shared__ float s_wt[CD > 0 ? NB : 1][CD > 0 ? NT : 1];  // alpha T of each listed pair
  __shared__ int s_item;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // selector bits and value index of the transposed row reductions
  const bool sel1 = lane & 4, sel2 = lane & 1, sel3 = lane & 2, sel4 = lane & 8;
  const int idx16 = 8 * ((lane >> 3) & 1) + 4 * ((lane >> 1) & 1) + 2 * (lane & 1) + ((lane >> 2) & 1);
  for (int idx = threadIdx.x; idx < NB * ACC; idx += NT) (&s_acc[0][0])[idx] = 0.f;
  int item = blockIdx.x;
  while (true) {
    if (PERSIST) {
      if (threadIdx.x == 0) s_item = (int)atomicAdd(&a.counters[CNT_QUEUE_BWD], 1ull);
      __syncthreads();
      item = s_item;
      __syncthreads();
    }
    if (item >= a.total_tiles) break;
    // persistent launches take the tiles in the order of tile_order (most
    // instances first), so the heaviest tiles do not form the tail
    const int tile = (PERSIST && a.tile_order) ? (int)a.tile_order[item] : item;
    const int v = view_of_tile(a.cams, a.V, tile);
    const CamDev& cam = a.cams[v];
    const int local = tile - cam.tile_base;
    const int ty = local / cam.ntx, tx = local - ty * cam.ntx;
    PixelBlock<TW, TH, 1> pb;
    pb.init(cam, tx, ty);
    float T = 1.f;
    bool done = pb.pix[0] < 0;
    const int64_t pxi = cam.pix_base + (done ? 0 : pb.pix[0]);
    const float G0 = done ? 0.f : a.dL[3 * pxi + 0];
    const float G1 = done ? 0.f : a.dL[3 * pxi + 1];
    const float G2 = done ? 0.f : a.dL[3 * pxi + 2];
    // colour of everything behind the instances blended so far: the final
    // colour minus their contributions
    float B0 = done ? 0.f : a.images_in[3 * pxi + 0];
    float B1 = done ? 0.f : a.images_in[3 * pxi + 1];
    float B2 = done ? 0.f : a.images_in[3 * pxi + 2];
    const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
    for (uint32_t b0 = start; b0 < end; b0 += NB) {
      const int nb = (int)min((uint32_t)NB, end - b0);
      if (threadIdx.x < NB * NW) (&s_cnt[0][0])[threadIdx.x] = 0u;
      if constexpr (CD > 0)
        stage_batch<N, NT, NB, CD>(S, a, v, b0, nb, &CS);
      else
        stage_batch<N, NT, NB>(S, a, v, b0, nb);
      // ---------------- phase 1: pixels ----------------
      // One instance for this thread's pixel.  `cached`: the integral comes
      // from the forward's store (ahc) instead of the density MLP.
      auto pixel_step = [&](const int j, const bool cached, const float ahc) {
        const int4 rc = S.rect[j];
        if (rc.y < pb.wx0 || rc.x > pb.wx1 || rc.w < pb.wy0 || rc.z > pb.wy1) return;  // wave-uniform
        const float4 r0 = S.rec[j][0], r1 = S.rec[j][1], r2 = S.rec[j][2];
        const float4 r3 = S.rec[j][3], r4 = S.rec[j][4], r5 = S.rec[j][5];
        PairGeom g;
        const bool gh = pair_geom(r0, r1, r2, r3, r4, r5, pb.pxc[0], pb.pyc[0], g, disc_coef_of(S, a, v, j));
        const bool hit = !done && gh;
        if (__ballot(hit) == 0) return;  // wave-uniform
        float ahat, QB = 0.f;  // QB = Q + b2 (recomputed path only)
        if (cached) {
          ahat = ahc;
        } else {
          const float* tabf = reinterpret_cast<const float*>(S.tab[j]);
          float Q = 0.f;
#pragma unroll 4
          for (int k = 0; k < N; ++k) {
            const float4 w = S.tab[j][k];
            const float w2 = tabf[4 * N + k];
            const float ph = __builtin_fmaf(w.x, g.p0, __builtin_fmaf(w.y, g.p1, __builtin_fmaf(w.z, g.p2, w.w)));
            const float hv = __builtin_fmaf(w.x, g.e0, __builtin_fmaf(w.y, g.e1, w.z * g.e2));
            const float c = cos_rev(ph);
            const float sn = sinc_rev(sin_rev(hv), hv);
            Q = __builtin_fmaf(w2 * c, sn, Q);
          }
          QB = Q + tabf[5 * N];
          ahat = 2.f * pb.L[0] * g.H * QB;
        }
        // the pair's colour (the per-ray network's, as in the forward)
        float c0 = r2.w, c1 = r3.w, c2 = r4.w;
        if constexpr (CD > 0) {
          float sg[3];
          const float iL = fast_rcp(pb.L[0]);
          ray_colour<CD>(reinterpret_cast<const float*>(CS.t[j]), reinterpret_cast<const float*>(CS.b[j]),
                         g.p0 - g.e0, g.p1 - g.e1, g.p2 - g.e2, g.d0 * iL, g.d1 * iL, g.d2 * iL, sg);
          c0 += sg[0];
          c1 += sg[1];
          c2 += sg[2];
        }
        // Without branches: a lane whose pixel does not blend this pair (a
        // miss, a terminated pixel, an alpha_min skip) takes alpha = 0, which
        // leaves T, the behind colour and every sum exactly as they were
        // (T < t_eps can only hold after the pair that set done).
        const float al0 = alpha_of(ahat, a.alpha_max);
        const bool blend = hit && !(a.alpha_min > 0.f && al0 < a.alpha_min);
        const float al = blend ? al0 : 0.f;
        const float wt = al * T;
        const float gc0 = G0 * wt, gc1 = G1 * wt, gc2 = G2 * wt;
        B0 = __builtin_fmaf(-c0, wt, B0);
        B1 = __builtin_fmaf(-c1, wt, B1);
        B2 = __builtin_fmaf(-c2, wt, B2);
        const float ta = T * (1.f - al);
        // live: positive, unclamped integral
        const bool gl = blend && ahat > 0.f && al < a.alpha_max;
        const float G = G0 * (c0 * ta - B0) + G1 * (c1 * ta - B1) + G2 * (c2 * ta - B2);
        const float wq = gl ? G * 2.f * pb.L[0] * g.H : 0.f;  // d loss / d Q
        // d loss / d H (direct) = G 2 L (Q + b2); from the stored integral
        // alpha-hat = 2 L H (Q + b2) when cached (H > 0 for a hit)
        const float gH = gl ? (cached ? G * ahat * fast_rcp(g.H) : G * 2.f * pb.L[0] * QB) : 0.f;
        // with the per-ray colour every blending pair is listed: its colour
        // gradient is G_c alpha T
        const bool live = (CD > 0 && al > 0.f) || wq != 0.f || gH != 0.f;
        T = ta;
        done = done || T < a.t_eps;
        // colour gradient: one transposed reduction of the three sums (with
        // the per-ray colour, phase 2 sums it)
        if constexpr (CD == 0) {
          const float z = nb_level<kDppRor8>(nb_level<kDppXor2>(
              tb_level<kDppXor1>(tb_level<kDppHalfMirror>(gc0, gc1, sel1), tb_level<kDppHalfMirror>(gc2, 0.f, sel1), sel2)));
          const int i4 = idx16 & 3;
          if (!sel3 && !sel4 && i4 < 3) atomicAdd(s_acc[j] + TS + 18 + i4, z);
        }
        // each wave appends to its own 64 slots of the instance's list (a
        // wave meets an instance once per batch), so no atomic is needed
        const unsigned long long lm = __ballot(live);
        if (lm) {
          if (live) {
            // slot: the number of live lanes below this one (mbcnt)
            const uint32_t pos =
                wave * 64 + __builtin_amdgcn_mbcnt_hi((uint32_t)(lm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)lm, 0u));
            s_pix[j][pos] = (PixIndex)pb.loc[0];
            s_wq[j][pos] = wq;
            s_gh[j][pos] = gH;
            if constexpr (CD > 0) s_wt[j][pos] = wt;
          }
          if (lane == 0) s_cnt[j][wave] = (uint32_t)__popcll(lm);
        }
      };
      if (a.ahat_cache && (int64_t)(b0 + nb) <= a.cache_instances) {
        // the forward's integrals of this batch, fetched together (only for
        // instances whose rectangle meets this wave's pixels)
        float pre[NB];
        const float* cp = a.ahat_cache + (int64_t)b0 * NT + pb.loc[0];
        const bool wave_live = __ballot(!done) != 0;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          pre[j] = 0.f;
          if (j < nb && wave_live) {
            const int4 rc = S.rect[j];
            if (!(rc.y < pb.wx0 || rc.x > pb.wx1 || rc.w < pb.wy0 || rc.z > pb.wy1)) pre[j] = cp[(int64_t)j * NT];
          }
        }
#pragma unroll
        for (int j = 0; j < NB; ++j)
          if (j < nb) pixel_step(j, true, pre[j]);
      } else {
        for (int j = 0; j < nb; ++j) pixel_step(j, false, 0.f);
      }
      __syncthreads();
      // ---------------- phase 2: live pairs ----------------
      int it = 0;
      for (int j = 0; j < nb; ++j) {
        // the list is the waves' regions in order: entry e lies in region w
        // with wstart[w] <= e < wstart[w + 1], at slot 64 w + e - wstart[w]
        uint32_t wstart[NW + 1];
        wstart[0] = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) wstart[w + 1] = wstart[w] + s_cnt[j][w];
        const uint32_t cnt = wstart[NW];
        for (uint32_t c0 = 0; c0 < cnt; c0 += 64, ++it) {
          if (it % NW != wave) continue;  // wave-uniform
          const uint32_t e = c0 + lane;
          const bool act = e < cnt;
          uint32_t slot = e;
#pragma unroll
          for (int w = 1; w < NW; ++w)
            if (e >= wstart[w]) slot = 64 * w + (e - wstart[w]);
          slot = act ? slot : 0;
          const int pix = act ? s_pix[j][slot] : 0;
          float wq = act ? s_wq[j][slot] : 0.f;
          float gHd = act ? s_gh[j][slot] : 0.f;
          const float pxc = (float)(tx * TW + pix % TW) + 0.5f;
          const float pyc = (float)(ty * TH + pix / TW) + 0.5f;
          const float4 r0 = S.rec[j][0], r1 = S.rec[j][1], r2 = S.rec[j][2];
          const float4 r3 = S.rec[j][3], r4 = S.rec[j][4], r5 = S.rec[j][5];
          PairGeom G;
          const double* dqj = disc_coef_of(S, a, v, j);
          const bool gh = pair_geom<true>(r0, r1, r2, r3, r4, r5, pxc, pyc, G, dqj);
          if (!gh) {  // float64 discriminant says the ray misses: no gradient
            wq = 0.f;
            gHd = 0.f;
          }
          const float sq_pair = G.sq;  // kept through the unit loop (the rest is recomputed)
          float wtp = 0.f;  // alpha T of the pair (per-ray colour)
          if constexpr (CD > 0) wtp = (act && gh) ? s_wt[j][slot] : 0.f;
          const float4* tab = S.tab[j];
          const float* tabf = reinterpret_cast<const float*>(S.tab[j]);
          float* acc = s_acc[j];
          float gp0 = 0.f, gp1 = 0.f, gp2 = 0.f, ge0 = 0.f, ge1 = 0.f, ge2 = 0.f;
          // Units in groups of eight (four when N = 4), one unit pair per
          // iteration.  A pair's eight terms (sWx, sWy, sWz, gph of both units)
          // take three transposed row levels and its two sW2 terms one; the
          // second pair of four units completes a 16-value row reduction
          // (lane: term 2 b1 + b0 of unit 2 b3 + b2), and the last pair of a
          // group finishes the sums across the rows with the row swaps, after
          // which each LDS address receives exactly one lane's sum.  y_prev,
          // s_prev carry the previous pair, z_prev, q_prev the previous four units.
          constexpr int GU = N >= 8 ? 8 : 4;
          const int tl = 2 * ((lane >> 1) & 1) + (lane & 1);         // term of this lane
          const int ul = 2 * ((lane >> 3) & 1) + ((lane >> 2) & 1);  // unit in its group of four
          float y_prev = 0.f, s_prev = 0.f, z_prev = 0.f, q_prev = 0.f;
#pragma unroll 1
          for (int k0 = 0; k0 < N; k0 += 2) {
            float v8[8], v2[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
              const int k = k0 + u;
              const float4 w = tab[k];
              const float w2 = tabf[4 * N + k];
              const float ph = __builtin_fmaf(w.x, G.p0, __builtin_fmaf(w.y, G.p1, __builtin_fmaf(w.z, G.p2, w.w)));
              const float hv = __builtin_fmaf(w.x, G.e0, __builtin_fmaf(w.y, G.e1, w.z * G.e2));
              const float c = cos_rev(ph), s = sin_rev(ph);
              const float sh = sin_rev(hv), ch = cos_rev(hv);
              const float rh = fast_rcp(hv);
              const float sn = fminf(sh * rh, kTwoPi);  // sinc, as in sinc_rev
              // d sn / d hv / (-2 pi): both phase derivatives below carry the
              // common factor -2 pi, applied once to their sums instead
              const float series = hv * __builtin_fmaf(kDsnC3n, hv * hv, kDsnC1n);
              const float general = __builtin_fmaf(sn, kInvTwoPi, -ch) * rh;
              const float dsn = fabsf(hv) < 0.02f ? series : general;
              const float wsn = wq * sn;
              const float gph = wsn * w2 * s;       // d loss / d ph / (-2 pi)
              const float ghv = wq * w2 * c * dsn;  // d loss / d hv / (-2 pi)
              v8[0 + u] = __builtin_fmaf(gph, G.p0, ghv * G.e0);
              v8[2 + u] = __builtin_fmaf(gph, G.p1, ghv * G.e1);
              v8[4 + u] = __builtin_fmaf(gph, G.p2, ghv * G.e2);
              v8[6 + u] = gph;
              v2[u] = wsn * c;
              gp0 = __builtin_fmaf(gph, w.x, gp0);
              gp1 = __builtin_fmaf(gph, w.y, gp1);
              gp2 = __builtin_fmaf(gph, w.z, gp2);
              ge0 = __builtin_fmaf(ghv, w.x, ge0);
              ge1 = __builtin_fmaf(ghv, w.y, ge1);
              ge2 = __builtin_fmaf(ghv, w.z, ge2);
            }
            const float x0 = tb_level<kDppXor1>(tb_level<kDppHalfMirror>(v8[0], v8[1], sel1),
                                                tb_level<kDppHalfMirror>(v8[2], v8[3], sel1), sel2);
            const float x1 = tb_level<kDppXor1>(tb_level<kDppHalfMirror>(v8[4], v8[5], sel1),
                                                tb_level<kDppHalfMirror>(v8[6], v8[7], sel1), sel2);
            const float y = tb_level<kDppXor2>(x0, x1, sel3);
            const float s2 = tb_level<kDppHalfMirror>(v2[0], v2[1], sel1);
            const int pi = (k0 >> 1) & (GU / 2 - 1);  // pair within the group (wave-uniform)
            if ((pi & 1) == 0) {
              y_prev = y;
              s_prev = s2;
              continue;
            }
            const float z = tb_level<kDppRor8>(y_prev, y, sel4);
            const float q = tb_level<kDppXor1>(s_prev, s2, sel2);  // unit 2 b0 + b2 of the four
            const int g = k0 & ~(GU - 1);
            if (GU == 8 && pi == 1) {
              z_prev = z;
              q_prev = q;
              continue;
            }
            if (GU == 8) {
              const float zz = cross_rows_pair(z_prev, z);  // rows 0, 1: first four units; rows 2, 3: second
              if ((lane & 16) == 0) atomicAdd(acc + 4 * (g + 4 * (lane >> 5) + ul) + tl, zz);
              const float q8 = cross_rows_sum(nb_level<kDppRor8>(tb_level<kDppXor2>(q_prev, q, sel3)));
              if (lane < 8) atomicAdd(acc + 4 * N + g + (idx16 & 7), q8);
            } else {
              const float zz = cross_rows_sum(z);
              if (lane < 16) atomicAdd(acc + 4 * (g + ul) + tl, zz);
              const float q4 = cross_rows_sum(nb_level<kDppRor8>(nb_level<kDppXor2>(q)));
              if (lane < 8 && !sel3) atomicAdd(acc + 4 * N + g + (idx16 & 3), q4);
            }
          }
          // The colour network's adjoint (per-ray colour) comes first, while
          // only p', e' and sqrt(disc) of the geometry are live, so that the
          // network's registers and the chain's are not live together: its
          // entry point is u = p' - e', its direction n = d' / L.
          float gn[3] = {0.f, 0.f, 0.f}, gu[3] = {0.f, 0.f, 0.f}, iLp = 0.f;
          int zz = 0;  // orders the re-reads of the record after the adjoint
          if constexpr (CD > 0) {
            iLp = 1.f / ray_length(cam, pxc, pyc);
            const float4 q0 = S.rec[j][0], q1 = S.rec[j][1], q2 = S.rec[j][2];
            const float ddx = pxc - q0.w, ddy = pyc - q1.w;
            const float n0 = __builtin_fmaf(q2.x, ddy, __builtin_fmaf(q1.x, ddx, q0.x)) * iLp;
            const float n1 = __builtin_fmaf(q2.y, ddy, __builtin_fmaf(q1.y, ddx, q0.y)) * iLp;
            const float n2 = __builtin_fmaf(q2.z, ddy, __builtin_fmaf(q1.z, ddx, q0.z)) * iLp;
            // the pair's pixel in the view (inactive lanes read the tile's
            // first pixel, which lies in the image, and carry wtp = 0)
            const int64_t gpx =
                cam.pix_base + (int64_t)(ty * TH + pix / TW) * cam.width + (tx * TW + pix % TW);
            const uint32_t pid = __builtin_amdgcn_readfirstlane(S.id[j]);
            ray_net_adjoint<CD>(reinterpret_cast<const float*>(CS.t[j]), reinterpret_cast<const float*>(CS.b[j]),
                                G.p0 - G.e0, G.p1 - G.e1, G.p2 - G.e2, n0, n1, n2, a.dL[3 * gpx + 0] * wtp,
                                a.dL[3 * gpx + 1] * wtp, a.dL[3 * gpx + 2] * wtp,
                                a.gctab + (int64_t)pid * RayColourLayout<16, CD>::CTS,
                                a.gcbias + ((int64_t)v * a.P + pid) * 16, acc + TS + 18, lane, idx16, sel1, sel2,
                                sel3, sel4, gu, gn);
            zz = zero_after(gu[0] + gn[0]);
          }
          // chain p', e', H -> d', m' -> record coefficients.  d' and m' are
          // recomputed from LDS here (the barrier keeps the compiler from
          // reusing the first computation), so only p', e' and sqrt(disc) stay
          // live through the unit loop.  The unit sums above are d loss / d ph
          // and d loss / d hv divided by -2 pi.
          asm volatile("" ::: "memory");
          {
            const float4 q0 = S.rec[j][0 + zz], q1 = S.rec[j][1 + zz], q2 = S.rec[j][2 + zz];
            const float4 q3 = S.rec[j][3 + zz], q4 = S.rec[j][4 + zz], q5 = S.rec[j][5 + zz];
            pair_dm(q0, q1, q2, q3, q4, q5, pxc, pyc, G);
            G.rA = fast_rcp(G.A);
            G.sq = sq_pair;
            G.H = G.sq * G.rA;
          }
          gp0 *= -kTwoPi;
          gp1 *= -kTwoPi;
          gp2 *= -kTwoPi;
          ge0 *= -kTwoPi;
          ge1 *= -kTwoPi;
          ge2 *= -kTwoPi;
          if constexpr (CD > 0) {
            gp0 += gu[0];
            gp1 += gu[1];
            gp2 += gu[2];
            ge0 -= gu[0];
            ge1 -= gu[1];
            ge2 -= gu[2];
          }
          float R[18];
#pragma unroll
          for (int r = 0; r < 18; ++r) R[r] = 0.f;
          if (wq != 0.f || gHd != 0.f || wtp != 0.f) {
            const float gHt = gHd + ge0 * G.d0 + ge1 * G.d1 + ge2 * G.d2;
            float gd0 = __builtin_fmaf(gn[0], iLp, ge0 * G.H), gd1 = __builtin_fmaf(gn[1], iLp, ge1 * G.H),
                  gd2 = __builtin_fmaf(gn[2], iLp, ge2 * G.H);
            const float gX0 = gp0 * G.rA, gX1 = gp1 * G.rA, gX2 = gp2 * G.rA;
            const float gA_p = -(gp0 * G.p0 + gp1 * G.p1 + gp2 * G.p2) * G.rA;
            const float gdisc = gHt * G.rA * 0.5f * fast_rcp(G.sq);
            const float gA = gdisc - gHt * G.H * G.rA + gA_p;
            const float gM = -gdisc;
            gd0 += 2.f * gA * G.d0 + (G.m1 * gX2 - G.m2 * gX1);
            gd1 += 2.f * gA * G.d1 + (G.m2 * gX0 - G.m0 * gX2);
            gd2 += 2.f * gA * G.d2 + (G.m0 * gX1 - G.m1 * gX0);
            const float gm0 = 2.f * gM * G.m0 + (gX1 * G.d2 - gX2 * G.d1);
            const float gm1 = 2.f * gM * G.m1 + (gX2 * G.d0 - gX0 * G.d2);
            const float gm2 = 2.f * gM * G.m2 + (gX0 * G.d1 - gX1 * G.d0);
            R[0] = gd0;
            R[1] = gd1;
            R[2] = gd2;
            R[3] = gd0 * G.dx;
            R[4] = gd1 * G.dx;
            R[5] = gd2 * G.dx;
            R[6] = gd0 * G.dy;
            R[7] = gd1 * G.dy;
            R[8] = gd2 * G.dy;
            R[9] = gm0;
            R[10] = gm1;
            R[11] = gm2;
            R[12] = gm0 * G.dx;
            R[13] = gm1 * G.dx;
            R[14] = gm2 * G.dx;
            R[15] = gm0 * G.dy;
            R[16] = gm1 * G.dy;
            R[17] = gm2 * G.dy;
          }
          {
            // record coefficients 0..15: one full transposed reduction
            float x4[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
              x4[q] = tb_level<kDppXor1>(tb_level<kDppHalfMirror>(R[4 * q], R[4 * q + 1], sel1),
                                         tb_level<kDppHalfMirror>(R[4 * q + 2], R[4 * q + 3], sel1), sel2);
            const float z = cross_rows_sum(tb_level<kDppRor8>(tb_level<kDppXor2>(x4[0], x4[1], sel3),
                                                              tb_level<kDppXor2>(x4[2], x4[3], sel3), sel4));
            if (lane < 16) atomicAdd(acc + TS + idx16, z);
            // coefficients 16, 17 and the b2 gradient (sum of d loss / d Q)
            const float t4 = cross_rows_sum(nb_level<kDppRor8>(nb_level<kDppXor2>(
                tb_level<kDppXor1>(tb_level<kDppHalfMirror>(R[16], R[17], sel1),
                                   tb_level<kDppHalfMirror>(wq, 0.f, sel1), sel2))));
            const int i4 = idx16 & 3;
            if (lane < 8 && !sel3 && i4 < 3) atomicAdd(i4 == 2 ? acc + 5 * N : acc + TS + 16 + i4, t4);
          }
        }
      }
      // flush the batch's accumulators to HBM (one float atomic per nonzero
      // value, spread over the workgroup) and clear them
      __syncthreads();
      for (int idx = threadIdx.x; idx < nb * ACC; idx += NT) {
        const int jj = idx / ACC, cc = idx - jj * ACC;
        float* slot = &s_acc[jj][cc];
        float val = *slot;
        if (val != 0.f) {
          const uint32_t p = S.id[jj];
          if (cc < 4 * N) val *= -kTwoPi;  // the phase-derivative sums (see the unit loop)
          if (cc < TS)
            atomic_add_f32(a.gtable + (int64_t)p * TS + cc, val);
          else
            atomic_add_f32(a.gview + ((int64_t)v * a.P + p) * kGViewFloats + (cc - TS), val);
          *slot = 0.f;
        }
      }
      if (__syncthreads_and(done)) break;
    }
    if (!PERSIST) break;
  }
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
struct TileShape {
  int tw, th, ppl;
};
static const TileShape kShapes[] = {{16, 16, 1}, {16, 16, 2}, {16, 16, 4}, {8, 8, 1}, {32, 16, 2}, {32, 16, 4}};
static const int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

int supported_tiles(int32_t* triples, int32_t max) {
  for (int i = 0; i < kNumShapes && i < max; ++i) {
    triples[3 * i] = kShapes[i].tw;
    triples[3 * i + 1] = kShapes[i].th;
    triples[3 * i + 2] = kShapes[i].ppl;
  }
  return kNumShapes;
}

bool tile_supported(int tw, int th, int ppl) {
  for (int i = 0; i < kNumShapes; ++i)
    if (kShapes[i].tw == tw && kShapes[i].th == th && kShapes[i].ppl == ppl) return true;
  return false;
}

// instances per backward batch for a tile shape; 0 picks the default
int bwd_batch_default(int tw, int th) { return tw * th >= 512 ? 4 : (tw * th >= 256 ? 8 : 16); }

bool bwd_batch_supported(int tw, int th, int nb) {
  if (tw == 16 && th == 16) return nb == 4 || nb == 8 || nb == 16;
  if (tw == 8 && th == 8) return nb == 16 || nb == 32;
  if (tw == 32 && th == 16) return nb == 4 || nb == 8;
  return false;
}

template <typename K>
static int persistent_grid(K kernel, int threads, int total) {
  int dev = 0, cus = 0, occ = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, threads, 0);
  if (occ < 1) occ = 1;
  int g = cus * occ;
  if (g > total) g = total;
  return g < 1 ? 1 : g;
}

template <int N, int TW, int TH, int PPL, int CD = 0>
static hipError_t fwd_shape(const RasterArgs& a, bool persist, bool count, hipStream_t st) {
  constexpr int NT = TW * TH / PPL;
  if (a.total_tiles <= 0) return hipSuccess;
  if (persist) {
    if (count) {
      auto k = render_fwd_kernel<N, TW, TH, PPL, true, true, CD>;
      hipLaunchKernelGGL(k, dim3(persistent_grid(k, NT, a.total_tiles)), dim3(NT), 0, st, a);
    } else {
      auto k = render_fwd_kernel<N, TW, TH, PPL, true, false, CD>;
      hipLaunchKernelGGL(k, dim3(persistent_grid(k, NT, a.total_tiles)), dim3(NT), 0, st, a);
    }
  } else {
    if (count)
      hipLaunchKernelGGL((render_fwd_kernel<N, TW, TH, PPL, false, true, CD>), dim3(a.total_tiles), dim3(NT), 0, st,
                         a);
    else
      hipLaunchKernelGGL((render_fwd_kernel<N, TW, TH, PPL, false, false, CD>), dim3(a.total_tiles), dim3(NT), 0,
                         st, a);
  }
  return hipGetLastError();
}

template <int TW, int TH, int PPL>
static hipError_t fwd_gauss_shape(const RasterArgs& a, bool persist, bool count, hipStream_t st) {
  constexpr int NT = TW * TH / PPL;
  if (a.total_tiles <= 0) return hipSuccess;
  if (persist) {
    if (count) {
      auto k = render_fwd_gauss_kernel<TW, TH, PPL, true, true>;
      hipLaunchKernelGGL(k, dim3(persistent_grid(k, NT, a.total_tiles)), dim3(NT), 0, st, a);
    } else {
      auto k = render_fwd_gauss_kernel<TW, TH, PPL, true, false>;
      hipLaunchKernelGGL(k, dim3(persistent_grid(k, NT, a.total_tiles)), dim3(NT), 0, st, a);
    }
  } else {
    if (count)
      hipLaunchKernelGGL((render_fwd_gauss_kernel<TW, TH, PPL, false, true>), dim3(a.total_tiles), dim3(NT), 0, st, a);
    else
      hipLaunchKernelGGL((render_fwd_gauss_kernel<TW, TH, PPL, false, false>), dim3(a.total_tiles), dim3(NT), 0, st,
                         a);
  }
  return hipGetLastError();
}

template <int N, int TW, int TH, int NB, int CD = 0>
static hipError_t bwd_shape(const RasterArgs& a, bool persist, hipStream_t st) {
  constexpr int NT = TW * TH;
  if (a.total_tiles <= 0) return hipSuccess;
  if (persist) {
    auto k = render_bwd_kernel<N, TW, TH, NB, true, CD>;
    hipLaunchKernelGGL(k, dim3(persistent_grid(k, NT, a.total_tiles)), dim3(NT), 0, st, a);
  } else {
    hipLaunchKernelGGL((render_bwd_kernel<N, TW, TH, NB, false, CD>), dim3(a.total_tiles), dim3(NT), 0, st, a);
  }
  return hipGetLastError();
}

// The per-ray colour network (colour mode 4) is built for N = 8 and 16,
// 16 x 16 tiles with one pixel per thread and backward batches of 8.
bool ray_colour_raster_supported(int N, int tw, int th, int ppl, int nb) {
  return (N == 8 || N == 16) && tw == 16 && th == 16 && ppl == 1 && (nb == 0 || nb == 8);
}

// one hidden layer (the kernels are written for two as well, but the
// adjoint of the 16 x 16 layer does not fit the register file)
template <int N>
static hipError_t fwd_ray(const RasterArgs& a, int cd, bool persist, bool count, hipStream_t st) {
  if (cd == 1) return fwd_shape<N, 16, 16, 1, 1>(a, persist, count, st);
  return hipErrorInvalidValue;
}

template <int N>
static hipError_t bwd_ray(const RasterArgs& a, int cd, bool persist, hipStream_t st) {
  if (cd == 1) return bwd_shape<N, 16, 16, 8, 1>(a, persist, st);
  return hipErrorInvalidValue;
}

template <int N>
static hipError_t fwd_n(const RasterArgs& a, int tw, int th, int ppl, bool persist, bool count, hipStream_t st) {
  if (tw == 16 && th == 16 && ppl == 1) return fwd_shape<N, 16, 16, 1>(a, persist, count, st);
  if (tw == 16 && th == 16 && ppl == 2) return fwd_shape<N, 16, 16, 2>(a, persist, count, st);
  if (tw == 16 && th == 16 && ppl == 4) return fwd_shape<N, 16, 16, 4>(a, persist, count, st);
  if (tw == 8 && th == 8 && ppl == 1) return fwd_shape<N, 8, 8, 1>(a, persist, count, st);
  if (tw == 32 && th == 16 && ppl == 2) return fwd_shape<N, 32, 16, 2>(a, persist, count, st);
  if (tw == 32 && th == 16 && ppl == 4) return fwd_shape<N, 32, 16, 4>(a, persist, count, st);
  return hipErrorInvalidValue;
}

template <int N>
static hipError_t bwd_n(const RasterArgs& a, int tw, int th, int nb, bool persist, hipStream_t st) {
  if (tw == 16 && th == 16 && nb == 4) return bwd_shape<N, 16, 16, 4>(a, persist, st);
  if (tw == 16 && th == 16 && nb == 8) return bwd_shape<N, 16, 16, 8>(a, persist, st);
  if (tw == 16 && th == 16 && nb == 16) return bwd_shape<N, 16, 16, 16>(a, persist, st);
  if (tw == 8 && th == 8 && nb == 16) return bwd_shape<N, 8, 8, 16>(a, persist, st);
  if (tw == 8 && th == 8 && nb == 32) return bwd_shape<N, 8, 8, 32>(a, persist, st);
  if (tw == 32 && th == 16 && nb == 4) return bwd_shape<N, 32, 16, 4>(a, persist, st);
  if (tw == 32 && th == 16 && nb == 8) return bwd_shape<N, 32, 16, 8>(a, persist, st);
  return hipErrorInvalidValue;
}

hipError_t launch_render_fwd(int N, int tw, int th, int ppl, bool persist, bool count, int cd, const RasterArgs& a,
                             hipStream_t st) {
  if (cd > 0) {
    if (!ray_colour_raster_supported(N, tw, th, ppl, 0)) return hipErrorInvalidValue;
    return N == 8 ? fwd_ray<8>(a, cd, persist, count, st) : fwd_ray<16>(a, cd, persist, count, st);
  }
  switch (N) {
    case 4: return fwd_n<4>(a, tw, th, ppl, persist, count, st);
    case 8: return fwd_n<8>(a, tw, th, ppl, persist, count, st);
    case 16: return fwd_n<16>(a, tw, th, ppl, persist, count, st);
    case 32: return fwd_n<32>(a, tw, th, ppl, persist, count, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_render_fwd_gauss(int tw, int th, int ppl, bool persist, bool count, const RasterArgs& a,
                                   hipStream_t st) {
  if (tw == 16 && th == 16 && ppl == 1) return fwd_gauss_shape<16, 16, 1>(a, persist, count, st);
  if (tw == 16 && th == 16 && ppl == 2) return fwd_gauss_shape<16, 16, 2>(a, persist, count, st);
  if (tw == 16 && th == 16 && ppl == 4) return fwd_gauss_shape<16, 16, 4>(a, persist, count, st);
  if (tw == 8 && th == 8 && ppl == 1) return fwd_gauss_shape<8, 8, 1>(a, persist, count, st);
  if (tw == 32 && th == 16 && ppl == 2) return fwd_gauss_shape<32, 16, 2>(a, persist, count, st);
  if (tw == 32 && th == 16 && ppl == 4) return fwd_gauss_shape<32, 16, 4>(a, persist, count, st);
  return hipErrorInvalidValue;
}

hipError_t launch_render_bwd(int N, int tw, int th, int nb, bool persist, int cd, const RasterArgs& a,
                             hipStream_t st) {
  if (cd > 0) {
    if (!ray_colour_raster_supported(N, tw, th, 1, nb)) return hipErrorInvalidValue;
    return N == 8 ? bwd_ray<8>(a, cd, persist, st) : bwd_ray<16>(a, cd, persist, st);
  }
  switch (N) {
    case 4: return bwd_n<4>(a, tw, th, nb, persist, st);
    case 8: return bwd_n<8>(a, tw, th, nb, persist, st);
    case 16: return bwd_n<16>(a, tw, th, nb, persist, st);
    case 32: return bwd_n<32>(a, tw, th, nb, persist, st);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// self test of the wave reduction (run by the test-suite on the device)
// ---------------------------------------------------------------------------
__global__ void wave_sum_selftest_kernel(const float* in, float* out) {
  const float v = in[blockIdx.x * 64 + threadIdx.x];
  const float t = wave_total(v);
  out[blockIdx.x * 64 + threadIdx.x] = t;
}

hipError_t launch_wave_sum_selftest(const float* in, float* out, int waves, hipStream_t st) {
  hipLaunchKernelGGL(wave_sum_selftest_kernel, dim3(waves), dim3(64), 0, st, in, out);
  return hipGetLastError();
}

}  // namespace snp
