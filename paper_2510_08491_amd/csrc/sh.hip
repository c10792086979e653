// Spherical-harmonics colour of degree 3 (the colour the paper adopts for
// novel-view synthesis, Sec. 3.1; four bands as in 3DGS, Sec. 3.3): per
// (primitive, view), with d = normalize(x_B - o_v) and the 16 real
// orthonormal harmonics Y_k of degrees 0..3 in (l, m) order (0,0), (1,-1),
// (1,0), (1,1), (2,-2) ... (3,3),
//
//     colour_c = max(0, 1/2 + sum_k Y_k(d) sh[k][c])
//
// Coefficients are stored per primitive as sh[16][3] (basis, channel).  In
// the dynamic-scene application the zero-order coefficient is a function of
// the time xi_t: sh[0][c] + sum_k tb_k sh_t[k][c] with tb = (xi, xi^2, xi^3,
// xi^4, cos xi, ..., cos 4 xi, sin xi, ..., sin 4 xi) (a polynomial and a
// Fourier series of degree 4).
#include "snp_internal.h"

namespace snp {

// normalisation constants of the real harmonics: 1/2 sqrt(1/pi), sqrt(3/(4pi)),
// 1/2 sqrt(15/pi), 1/4 sqrt(5/pi), 1/4 sqrt(15/pi), 1/4 sqrt(35/(2pi)),
// 1/2 sqrt(105/pi), 1/4 sqrt(21/(2pi)), 1/4 sqrt(7/pi), 1/4 sqrt(105/pi)
constexpr float kSh0 = 0.28209479177387814f;
constexpr float kSh1 = 0.4886025119029199f;
constexpr float kSh2a = 1.0925484305920792f;
constexpr float kSh2b = 0.31539156525252005f;
constexpr float kSh2c = 0.5462742152960396f;
constexpr float kSh3a = 0.5900435899266435f;
constexpr float kSh3b = 2.890611442640554f;
constexpr float kSh3c = 0.4570457994644658f;
constexpr float kSh3d = 0.3731763325901154f;
constexpr float kSh3e = 1.445305721320277f;

__device__ __forceinline__ void sh_basis(float x, float y, float z, float (&Y)[16]) {
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[0] = kSh0;
  Y[1] = kSh1 * y;
  Y[2] = kSh1 * z;
  Y[3] = kSh1 * x;
  Y[4] = kSh2a * x * y;
  Y[5] = kSh2a * y * z;
  Y[6] = kSh2b * (3.f * zz - 1.f);
  Y[7] = kSh2a * x * z;
  Y[8] = kSh2c * (xx - yy);
  Y[9] = kSh3a * y * (3.f * xx - yy);
  Y[10] = kSh3b * x * y * z;
  Y[11] = kSh3c * y * (5.f * zz - 1.f);
  Y[12] = kSh3d * z * (5.f * zz - 3.f);
  Y[13] = kSh3c * x * (5.f * zz - 1.f);
  Y[14] = kSh3e * z * (xx - yy);
  Y[15] = kSh3a * x * (xx - 3.f * yy);
}

// gradient with respect to (x, y, z) of sum_k w_k Y_k (the polynomials above)
__device__ __forceinline__ void sh_weighted_grad(float x, float y, float z, const float (&w)[16], float& gx, float& gy,
                                                 float& gz) {
  const float xx = x * x, yy = y * y, zz = z * z;
  gx = kSh1 * w[3] + kSh2a * (y * w[4] + z * w[7]) + 2.f * kSh2c * x * w[8] + 6.f * kSh3a * x * y * w[9] +
       kSh3b * y * z * w[10] + kSh3c * (5.f * zz - 1.f) * w[13] + 2.f * kSh3e * x * z * w[14] +
       3.f * kSh3a * (xx - yy) * w[15];
  gy = kSh1 * w[1] + kSh2a * (x * w[4] + z * w[5]) - 2.f * kSh2c * y * w[8] + 3.f * kSh3a * (xx - yy) * w[9] +
       kSh3b * x * z * w[10] + kSh3c * (5.f * zz - 1.f) * w[11] - 2.f * kSh3e * y * z * w[14] -
       6.f * kSh3a * x * y * w[15];
  gz = kSh1 * w[2] + kSh2a * (y * w[5] + x * w[7]) + 6.f * kSh2b * z * w[6] + kSh3b * x * y * w[10] +
       10.f * kSh3c * y * z * w[11] + kSh3d * (15.f * zz - 3.f) * w[12] + 10.f * kSh3c * x * z * w[13] +
       kSh3e * (xx - yy) * w[14];
}

__device__ __forceinline__ void view_dir(const ShArgs& a, int v, int64_t p, float& x, float& y, float& z) {
  const CamDev& cam = a.cams[v];
  const float dx = a.centers[3 * p] - cam.o_f[0];
  const float dy = a.centers[3 * p + 1] - cam.o_f[1];
  const float dz = a.centers[3 * p + 2] - cam.o_f[2];
  const float il = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
  x = dx * il;
  y = dy * il;
  z = dz * il;
}

// the zero-order coefficient of channel ch (time dependent with sh_t)
__device__ __forceinline__ float zero_order(const ShArgs& a, int64_t p, const float* c, int ch) {
  float s0 = c[ch];
  if (a.sh_t) {
    const float* t = a.sh_t + p * (kShTime * 3);
#pragma unroll
    for (int k = 0; k < kShTime; ++k) s0 = __builtin_fmaf(a.tb[k], t[3 * k + ch], s0);
  }
  return s0;
}

// one thread per (view, primitive): colour into the record
__global__ void __launch_bounds__(256) sh_fwd_kernel(ShArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)a.V * a.P || a.tile_counts[i] == 0) return;
  const int v = (int)(i / a.P);
  const int64_t p = i - (int64_t)v * a.P;
  float x, y, z, Y[16];
  view_dir(a, v, p, x, y, z);
  sh_basis(x, y, z, Y);
  const float* c = a.sh + p * kShCoeffs;
  float col[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    float s = 0.5f;
#pragma unroll
    for (int k = 1; k < 16; ++k) s = __builtin_fmaf(Y[k], c[3 * k + ch], s);
    s = __builtin_fmaf(Y[0], zero_order(a, p, c, ch), s);
    col[ch] = fmaxf(s, 0.f);
  }
  float* rec = a.records + i * kRecFloats;
  rec[11] = col[0];
  rec[15] = col[1];
  rec[19] = col[2];
}

// one thread per primitive, its views in turn: coefficient gradients summed
// over the views (kept in registers), the direction gradient of each view
// written to the view's gradient record (slots 21..23) for the chain to the
// centre; a clamped channel passes no gradient
__global__ void __launch_bounds__(128) sh_bwd_kernel(ShArgs a) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.P) return;
  float c[16][3], g[16][3];
#pragma unroll
  for (int k = 0; k < 16; ++k)
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      c[k][ch] = a.sh[p * kShCoeffs + 3 * k + ch];
      g[k][ch] = 0.f;
    }
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) c[0][ch] = zero_order(a, p, a.sh + p * kShCoeffs, ch);
  for (int v = 0; v < a.V; ++v) {
    const int64_t i = (int64_t)v * a.P + p;
    if (a.tile_counts[i] == 0) continue;
    float x, y, z, Y[16];
    view_dir(a, v, p, x, y, z);
    sh_basis(x, y, z, Y);
    float* gv = a.gview + i * kGViewFloats;
    float gc[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      float s = 0.5f;
#pragma unroll
      for (int k = 0; k < 16; ++k) s = __builtin_fmaf(Y[k], c[k][ch], s);
      gc[ch] = s > 0.f ? gv[18 + ch] : 0.f;
    }
    float w[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) g[k][ch] = __builtin_fmaf(gc[ch], Y[k], g[k][ch]);
      w[k] = gc[0] * c[k][0] + gc[1] * c[k][1] + gc[2] * c[k][2];
    }
    float gx, gy, gz;
    sh_weighted_grad(x, y, z, w, gx, gy, gz);
    gv[21] = gx;
    gv[22] = gy;
    gv[23] = gz;
  }
  if (a.g_sh) {
#pragma unroll
    for (int k = 0; k < 16; ++k)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) a.g_sh[p * kShCoeffs + 3 * k + ch] += g[k][ch];
  }
  // the time coefficients: d S0(xi) / d sh_t[k][c] = tb_k
  if (a.sh_t && a.g_sh_t) {
#pragma unroll
    for (int k = 0; k < kShTime; ++k)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) a.g_sh_t[p * (kShTime * 3) + 3 * k + ch] += a.tb[k] * g[0][ch];
  }
}

hipError_t launch_sh_fwd(const ShArgs& a, hipStream_t st) {
  const int64_t n = (int64_t)a.V * a.P;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(sh_fwd_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_sh_bwd(const ShArgs& a, hipStream_t st) {
  if (a.P <= 0) return hipSuccess;
  hipLaunchKernelGGL(sh_bwd_kernel, dim3((unsigned)((a.P + 127) / 128)), dim3(128), 0, st, a);
  return hipGetLastError();
}

}  // namespace snp
